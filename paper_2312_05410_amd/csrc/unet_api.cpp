// Host runtime of the time-conditioned U-Net (Materials and Methods, "U-Net
// with temporal conditioning"; "Training of the network"): parameter and
// workspace layout, the forward and backward schedules over the kernels of
// unet_conv.hip / unet_ops.hip, Adam, and the single-op entry points.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "pf.h"
#include "unet.h"
#include "unet_kernels.h"

namespace {

using namespace pfu;

// operand weight padding: K to a multiple of 32 (one wide MFMA step), output
// rows to a multiple of 128 (the widest block tile)
size_t r32(size_t v) { return (v + 31) / 32 * 32; }
size_t r128(size_t v) { return (v + 127) / 128 * 128; }
size_t r256(size_t v) { return (v + 255) / 256 * 256; }

bool cfg_ok(const unet_config* c)
{
    if (!c) return false;
    if (c->in_ch != 4 || c->out_ch != 3) return false;
    if (c->levels < 2 || c->levels > kMaxLevels || c->base < 8 || c->base % 8) return false;
    if (c->height <= 0 || c->width <= 0 || c->max_batch <= 0) return false;
    const int f = 1 << (c->levels - 1);
    if (c->height % f || c->width % f) return false;
    if ((long)c->max_batch * c->height * c->width > (1L << 30)) return false;
    const long top = (long)c->base << (c->levels - 1);
    if (top > 256) return false;  // normalisation blocks keep one channel per thread
    if (c->groups <= 0 || c->base % c->groups) return false;
    if (c->head_groups <= 0 || c->out_ch % c->head_groups) return false;
    if (c->mlp_hidden <= 0 || c->mlp_hidden > 256 || c->basis <= 0 || c->basis > 256) return false;
    if (!(c->gn_eps > 0.f)) return false;
    return true;
}

// Wgrad partial products: pixel chunks (multiples of 64, the staged
// kernel's step) chosen for about 1024 blocks.
int wgrad_chunk(long P, int taps, int Nout, int C1, int C2)
{
    const long tiles = wgrad_blocks_per_chunk(taps == 9 ? kConvFwd : kUpFwd, Nout, C1, C2);
    long chunks = std::max(1L, (1024 + tiles - 1) / tiles);
    chunks = std::min(chunks, std::max(1L, (P + 255) / 256));
    long ch = (P + chunks - 1) / chunks;
    ch = (ch + 63) / 64 * 64;
    return (int)std::max(64L, ch);
}
size_t wgrad_floats(long P, int taps, int Nout, int C1, int C2)
{
    const long ch = wgrad_chunk(P, taps, Nout, C1, C2);
    const long chunks = (P + ch - 1) / ch;
    return (size_t)chunks * taps * Nout * (C1 + C2);
}

// ------------------------------------------------------------------ plan
struct Conv {
    int pw = -1, pg = -1, pb = -1;  // parameter indices (weight, gamma, beta)
    int taps = 9, cin1 = 0, cin2 = 0, cout = 0, groups = 1, gelu = 1;
    bool folded = false;             // 4-channel input: forward operand [1][ldo_f][64], k = 4 tap + c
    uint16_t* wf = nullptr;          // BF16 forward operand [taps][ldo_f][ldk_f]
    uint16_t* wt = nullptr;          // BF16 transposed operand (input gradient)
    // at most 4 output channels: the input gradient's kFirst operand
    // [ldo_tk][64], k = 4 tap + c over the mirrored taps
    uint16_t* wtk = nullptr;
    int ldo_f = 0, ldk_f = 0, ldo_t = 0, ldk_t = 0, ldo_tk = 0;
};

struct Net {
    unet_config c{};
    int L = 0;
    int w[kMaxLevels] = {};
    std::vector<unet_param_desc> params;
    int64_t nparams = 0;
    Conv enc[kMaxLevels], mid, dec[kMaxLevels], head, up[kMaxLevels];  // up[l]: level l -> l-1
    int mlp[6] = {};                                                   // w0 b0 w1 b1 w2 b2
    int film[kMaxLevels] = {};

    int add(const char* name, std::initializer_list<int> dims)
    {
        unet_param_desc d{};
        snprintf(d.name, sizeof d.name, "%s", name);
        d.offset = nparams;
        d.count = 1;
        d.ndim = 0;
        for (int v : dims) {
            d.dims[d.ndim++] = v;
            d.count *= v;
        }
        nparams += d.count;
        params.push_back(d);
        return (int)params.size() - 1;
    }
    void add_conv(Conv& k, const char* pre, int cin1, int cin2, int cout, int groups, int gelu)
    {
        std::string p(pre);
        k.taps = 9;
        k.cin1 = cin1;
        k.cin2 = cin2;
        k.cout = cout;
        k.groups = groups;
        k.gelu = gelu;
        k.pw = add((p + ".w").c_str(), {9, cout, cin1 + cin2});
        k.pg = add((p + ".gamma").c_str(), {cout});
        k.pb = add((p + ".beta").c_str(), {cout});
    }

    explicit Net(const unet_config& cfg) : c(cfg)
    {
        L = c.levels;
        for (int l = 0; l < L; ++l) w[l] = c.base << l;
        char nm[32];
        for (int l = 0; l < L; ++l) {
            snprintf(nm, sizeof nm, "enc%d", l);
            add_conv(enc[l], nm, l ? w[l - 1] : c.in_ch, 0, w[l], c.groups, 1);
        }
        enc[0].folded = true;
        add_conv(mid, "mid", w[L - 1], 0, w[L - 1], c.groups, 1);
        for (int l = L - 1; l >= 1; --l) {
            snprintf(nm, sizeof nm, "up%d.w", l);
            up[l].taps = 1;
            up[l].cin1 = w[l];
            up[l].cout = w[l - 1];
            up[l].pw = add(nm, {4, w[l - 1], w[l]});
            if (l - 1 >= 0) {
                snprintf(nm, sizeof nm, "dec%d", l - 1);
                add_conv(dec[l - 1], nm, w[l - 1], w[l - 1], w[l - 1], c.groups, 1);
            }
        }
        add_conv(head, "head", w[0], 0, c.out_ch, c.head_groups, 0);
        const int Hd = c.mlp_hidden, F = c.basis;
        mlp[0] = add("mlp.w0", {Hd, 1});
        mlp[1] = add("mlp.b0", {Hd});
        mlp[2] = add("mlp.w1", {Hd, Hd});
        mlp[3] = add("mlp.b1", {Hd});
        mlp[4] = add("mlp.w2", {F, Hd});
        mlp[5] = add("mlp.b2", {F});
        for (int l = 0; l < L; ++l) {
            snprintf(nm, sizeof nm, "film%d.w", l);
            film[l] = add(nm, {w[l], F});
        }
    }
    long P(int l, int n) const { return (long)n * (c.height >> l) * (c.width >> l); }
};

// Device buffers, carved from one workspace by a bump allocator (a null
// base only measures).
struct Bufs {
    uint16_t* xin;
    float* y[kMaxLevels];
    uint16_t *z[kMaxLevels], *zs[kMaxLevels], *q[kMaxLevels];
    float* st[kMaxLevels];
    float* ym;
    uint16_t* am;
    float* stm;
    float* yd[kMaxLevels];
    uint16_t *ad[kMaxLevels], *d[kMaxLevels];
    float* std_[kMaxLevels];
    float *yh, *sth;
    float *jump, *h0, *h1, *f, *sc[kMaxLevels];
    uint32_t* mlpc;                 // [n][L][2]: jump bits and parameter generation of each sc[l][n]
    float* gcoef;                   // GN forward coefficients [2][n][C] (shared by every GN)
    float *mdf, *mdh1, *mdh0;
    // backward
    float* gout;
    uint16_t* dyh;
    float* dad[kMaxLevels];  // gradient of ad[l] (l = L-1: of am)
    uint16_t* dyd[kMaxLevels];
    uint16_t* dym;
    float* dzs[kMaxLevels];
    uint16_t* dd[kMaxLevels];
    uint16_t* dye[kMaxLevels];
    float *dq[kMaxLevels], *dz[kMaxLevels];
    float* ds[kMaxLevels];
    double *lpart, *loss;
    float* wpart;
    size_t wpart_floats;
    float* csum;
    double* cacc;
    size_t bytes;
};

struct Bump {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t count)
    {
        const size_t o = off;
        off = r256(off + count * sizeof(T));
        return base ? (T*)(base + o) : nullptr;
    }
};

void carve(Net& net, char* base, Bufs& b)
{
    Bump m{base};
    const unet_config& c = net.c;
    const int n = c.max_batch, L = net.L, Hd = c.mlp_hidden, F = c.basis;
    const int* w = net.w;
    b.xin = m.take<uint16_t>(net.P(0, n) * 4);
    size_t part = 0, csum = 0;
    int cmax = 0, gmax = 0;
    // 3x3 weight gradients: the staged kernel's partials or, where the shape
    // takes it, the halo-tile kernel's
    auto wg9 = [](long P, int Nout, int C1, int C2) {
        return std::max(wgrad_floats(P, 9, Nout, C1, C2), wgrad_halo_floats(Nout, C1, C2));
    };
    auto note_gn = [&](long P1, int C, int G) {
        // partials: the normalisation's own chunks, or one per conv tile (>= 64 pixels)
        csum = std::max(csum, std::max(gn_csum_floats(n, (int)P1, C), (size_t)n * ((P1 + 63) / 64) * C * 3));
        cmax = std::max(cmax, C);
        gmax = std::max(gmax, G);
    };
    for (int l = 0; l < L; ++l) {
        const long Pl = net.P(l, 1) * n;
        b.y[l] = m.take<float>(Pl * w[l]);
        b.z[l] = l < L - 1 ? m.take<uint16_t>(Pl * w[l]) : nullptr;
        b.zs[l] = m.take<uint16_t>(Pl * w[l]);
        b.q[l] = l < L - 1 ? m.take<uint16_t>(net.P(l + 1, n) * w[l]) : nullptr;
        b.st[l] = m.take<float>((size_t)n * c.groups * 2);
        b.sc[l] = m.take<float>((size_t)n * w[l]);
        b.ds[l] = m.take<float>((size_t)n * w[l]);
        b.dzs[l] = m.take<float>(Pl * w[l]);
        b.dye[l] = m.take<uint16_t>(Pl * w[l]);
        b.dq[l] = l < L - 1 ? m.take<float>(net.P(l + 1, n) * w[l]) : nullptr;
        b.dz[l] = l < L - 1 ? m.take<float>(Pl * w[l]) : nullptr;
        note_gn(net.P(l, 1), w[l], c.groups);
        const Conv& k = net.enc[l];
        part = std::max(part, wg9(Pl, k.cout, k.cin1, 0));
    }
    {
        const long Pm = net.P(L - 1, n);
        b.ym = m.take<float>(Pm * w[L - 1]);
        b.am = m.take<uint16_t>(Pm * w[L - 1]);
        b.stm = m.take<float>((size_t)n * c.groups * 2);
        b.dym = m.take<uint16_t>(Pm * w[L - 1]);
        b.dad[L - 1] = m.take<float>(Pm * w[L - 1]);
        part = std::max(part, wg9(Pm, w[L - 1], w[L - 1], 0));
    }
    for (int l = 0; l < L - 1; ++l) {
        const long Pl = net.P(l, n);
        b.yd[l] = m.take<float>(Pl * w[l]);
        b.ad[l] = m.take<uint16_t>(Pl * w[l]);
        b.d[l] = m.take<uint16_t>(Pl * w[l]);
        b.std_[l] = m.take<float>((size_t)n * c.groups * 2);
        b.dad[l] = m.take<float>(Pl * w[l]);
        b.dyd[l] = m.take<uint16_t>(Pl * w[l]);
        b.dd[l] = m.take<uint16_t>(Pl * w[l]);
        part = std::max(part, wg9(Pl, w[l], w[l], w[l]));
        part = std::max(part, wgrad_floats(net.P(l + 1, n), 1, 4 * w[l], w[l + 1], 0));
    }
    {
        const long P0 = net.P(0, n);
        b.yh = m.take<float>(P0 * c.out_ch);
        b.sth = m.take<float>((size_t)n * c.head_groups * 2);
        b.gout = m.take<float>(P0 * c.out_ch);
        b.dyh = m.take<uint16_t>(P0 * c.out_ch);
        note_gn(net.P(0, 1), c.out_ch, c.head_groups);
        part = std::max(part, wg9(P0, c.out_ch, w[0], 0));
    }
    b.jump = m.take<float>((size_t)n);
    b.mlpc = m.take<uint32_t>((size_t)n * L * 2);
    b.gcoef = m.take<float>((size_t)2 * n * std::max(w[L - 1], c.out_ch));
    b.h0 = m.take<float>((size_t)n * Hd);
    b.h1 = m.take<float>((size_t)n * Hd);
    b.f = m.take<float>((size_t)n * F);
    b.mdf = m.take<float>((size_t)n * F);
    b.mdh1 = m.take<float>((size_t)n * Hd);
    b.mdh0 = m.take<float>((size_t)n * Hd);
    b.lpart = m.take<double>(rel_mse_partial_doubles());
    b.loss = m.take<double>(4);
    b.wpart = m.take<float>(part);
    b.wpart_floats = part;
    b.csum = m.take<float>(csum);
    b.cacc = m.take<double>((size_t)n * (3 * cmax + 2 * gmax));
    // BF16 operand copies of every weight
    auto wcopies = [&](Conv& k, bool tr) {
        if (k.folded) {
            k.ldo_f = (int)r128(k.cout);
            k.ldk_f = 64;
            k.wf = m.take<uint16_t>((size_t)k.ldo_f * 64);
            return;
        }
        const int R = k.taps == 9 ? k.cout : 4 * k.cout, Kc = k.cin1 + k.cin2;
        k.ldo_f = (int)r128(R);
        k.ldk_f = (int)r32(Kc);
        k.wf = m.take<uint16_t>((size_t)k.taps * k.ldo_f * k.ldk_f);
        if (tr) {
            k.ldo_t = (int)r128(Kc);
            k.ldk_t = (int)r32(R);
            k.wt = m.take<uint16_t>((size_t)k.taps * k.ldo_t * k.ldk_t);
            if (k.taps == 9 && k.cout <= 4 && k.cin2 == 0) {
                k.ldo_tk = (int)r128(Kc);
                k.wtk = m.take<uint16_t>((size_t)k.ldo_tk * 64);
            }
        }
    };
    for (int l = 0; l < L; ++l) wcopies(net.enc[l], l > 0);
    wcopies(net.mid, true);
    for (int l = 1; l < L; ++l) wcopies(net.up[l], true);
    for (int l = 0; l < L - 1; ++l) wcopies(net.dec[l], true);
    wcopies(net.head, true);
    b.bytes = m.off;
}

}  // namespace

struct unet_handle {
    Net net;
    Bufs b{};
    float* params;
    float* grads;
    hipStream_t stream;
    int last_n = 0;
    uint32_t param_gen = 0;   // advanced whenever the parameters may have changed (never 0 after create)
    explicit unet_handle(const unet_config& c) : net(c) {}
};

namespace {

int dev_err(hipError_t e) { return e == hipSuccess ? PF_OK : PF_EDEVICE; }
#define UCHECK(x)                                     \
    do {                                              \
        hipError_t e_ = (x);                          \
        if (e_ != hipSuccess) return PF_EDEVICE;      \
    } while (0)

bool al(const void* p, size_t a) { return p && ((uintptr_t)p % a) == 0; }

float* par(unet_handle* h, int idx) { return h->params + h->net.params[idx].offset; }
float* grd(unet_handle* h, int idx) { return h->grads + h->net.params[idx].offset; }

// the operand copies of one convolution's weight
void prep_items(unet_handle* h, const Conv& k, std::vector<PrepItem>& v)
{
    PrepItem p{};
    p.W = par(h, k.pw);
    p.taps = k.taps;
    p.R = k.taps == 9 ? k.cout : 4 * k.cout;
    p.Kc = k.cin1 + k.cin2;
    if (k.folded) {
        p.kind = kPrepFirst;
        p.fwd = k.wf;
        p.ldo_f = k.ldo_f;
        v.push_back(p);
        return;
    }
    p.kind = kPrepPlain;
    p.fwd = k.wf;
    p.ldo_f = k.ldo_f;
    p.ldk_f = k.ldk_f;
    p.tr = k.wt;
    p.ldo_t = k.ldo_t;
    p.ldk_t = k.ldk_t;
    v.push_back(p);
    if (k.wtk) {
        p.kind = kPrepFirstGrad;
        p.fwd = nullptr;
        p.tr = k.wtk;
        p.ldo_t = k.ldo_tk;
        v.push_back(p);
    }
}

int prepare_all(unet_handle* h)
{
    Net& net = h->net;
    // the time basis memo (sc[l][n] keyed by jump[n] and this generation)
    // is void from here on
    if (++h->param_gen == 0) h->param_gen = 1;
    // every weight's operand copies in one launch
    std::vector<PrepItem> v;
    for (int l = 0; l < net.L; ++l) prep_items(h, net.enc[l], v);
    prep_items(h, net.mid, v);
    for (int l = 1; l < net.L; ++l) prep_items(h, net.up[l], v);
    for (int l = 0; l < net.L - 1; ++l) prep_items(h, net.dec[l], v);
    prep_items(h, net.head, v);
    return dev_err(weight_prep_batch(v.data(), (int)v.size(), h->stream));
}

ConvArgs conv_args(const Conv& k, int n, int H, int W, const uint16_t* x1, const uint16_t* x2)
{
    ConvArgs a{};
    a.in1 = x1;
    a.in2 = x2;
    a.Wt = k.wf;
    a.N = n;
    a.H = H;
    a.W = W;
    a.C1 = k.cin1;
    a.C2 = k.cin2;
    a.Nout = k.taps == 9 ? k.cout : 4 * k.cout;
    a.O1 = a.Nout;
    a.ldk = k.ldk_f;
    a.ldo = k.ldo_f;
    return a;
}

// Input gradient of a 3x3 convolution: split into (dx1 f32, dx2 bf16).
ConvArgs dgrad_args(const Conv& k, int n, int H, int W, const uint16_t* dy)
{
    ConvArgs a{};
    a.in1 = dy;
    a.Wt = k.wt;
    a.N = n;
    a.H = H;
    a.W = W;
    a.C1 = k.cout;
    a.C2 = 0;
    a.Nout = k.cin1 + k.cin2;
    a.O1 = k.cin1;
    a.ldk = k.ldk_t;
    a.ldo = k.ldo_t;
    return a;
}

GNArgs gn_args(unet_handle* h, const Conv& k, int n, long P1, const float* y, float* stats)
{
    GNArgs g{};
    g.y = y;
    g.gamma = par(h, k.pg);
    g.beta = par(h, k.pb);
    g.stats = stats;
    g.csum = h->b.csum;
    g.cacc = h->b.cacc;
    g.N = n;
    g.P = (int)P1;
    g.C = k.cout;
    g.G = k.groups;
    g.gelu = k.gelu;
    g.eps = h->net.c.gn_eps;
    g.coef = h->b.gcoef;
    return g;
}

WgradArgs wgrad_args(unet_handle* h, int n, int H, int W, const uint16_t* dy, int Nout, const uint16_t* x1, int C1,
                     const uint16_t* x2, int C2, int taps)
{
    WgradArgs a{};
    a.dy = dy;
    a.x1 = x1;
    a.x2 = x2;
    a.partial = h->b.wpart;
    a.partial_cap = h->b.wpart_floats;
    a.N = n;
    a.H = H;
    a.W = W;
    a.C1 = C1;
    a.C2 = C2;
    a.Nout = Nout;
    a.chunk = wgrad_chunk((long)n * H * W, taps, Nout, C1, C2);
    return a;
}

MLPArgs mlp_args(unet_handle* h, int n, const float* jump)
{
    Net& net = h->net;
    MLPArgs a{};
    a.jump = jump;
    a.W0 = par(h, net.mlp[0]);
    a.b0 = par(h, net.mlp[1]);
    a.W1 = par(h, net.mlp[2]);
    a.b1 = par(h, net.mlp[3]);
    a.W2 = par(h, net.mlp[4]);
    a.b2 = par(h, net.mlp[5]);
    a.gW0 = grd(h, net.mlp[0]);
    a.gb0 = grd(h, net.mlp[1]);
    a.gW1 = grd(h, net.mlp[2]);
    a.gb1 = grd(h, net.mlp[3]);
    a.gW2 = grd(h, net.mlp[4]);
    a.gb2 = grd(h, net.mlp[5]);
    a.h0 = h->b.h0;
    a.h1 = h->b.h1;
    a.f = h->b.f;
    a.df = h->b.mdf;
    a.dh1 = h->b.mdh1;
    a.dh0 = h->b.mdh0;
    a.N = n;
    a.Hd = net.c.mlp_hidden;
    a.F = net.c.basis;
    a.L = net.L;
    a.cache = h->b.mlpc;
    a.gen = h->param_gen;
    for (int l = 0; l < net.L; ++l) {
        a.Wl[l] = par(h, net.film[l]);
        a.gWl[l] = grd(h, net.film[l]);
        a.sc[l] = h->b.sc[l];
        a.dsc[l] = h->b.ds[l];
        a.C[l] = net.w[l];
    }
    return a;
}

// Convolution whose output feeds a group normalisation: the wide kernel's
// epilogue writes the normalisation's partial sums when a sample's pixels
// split evenly into its blocks.
int conv_gn(unet_handle* h, ConvArgs a, int mode, GNArgs g, const MLPArgs* mlp = nullptr, float* jump_copy = nullptr)
{
    const int chunks = conv_stat_chunks(a, mode);
    if (chunks > 0) {
        a.gsum = h->b.csum;
        g.sums_ready = 1;
        g.chunks = chunks;
    }
    UCHECK(conv_gemm(a, mode, h->stream));
    UCHECK(gn_forward(g, h->stream, mlp, jump_copy));
    return PF_OK;
}

#define RCHECK(x)                      \
    do {                               \
        const int r_ = (x);            \
        if (r_ != PF_OK) return r_;    \
    } while (0)

// train: also keep what the backward pass reads (the unconditioned encoder
// latents z_l behind the pooling)
int forward(unet_handle* h, int n, const float* jump, const float* c, const float* phi, const float* rho, float* oc,
            float* ophi, float* orho, bool train)
{
    Net& net = h->net;
    Bufs& b = h->b;
    hipStream_t s = h->stream;
    const int L = net.L;
    auto Hl = [&](int l) { return net.c.height >> l; };
    auto Wl = [&](int l) { return net.c.width >> l; };
    const long P0 = net.P(0, 1);
    const MLPArgs mlp = mlp_args(h, n, jump);
    // inference: the first layer gathers its input from the state fields and
    // its normalisation launch also evaluates the time basis and the FiLM
    // scales (and copies the jumps); training keeps the assembled input for
    // the weight gradient, so input assembly, time basis and FiLM scales run
    // as one launch first.  Both copy the jumps, which the head's
    // normalisation and the backward pass read.
    const bool fused = !train && mlp_fused_ok(mlp);
    if (!fused) UCHECK(prologue_forward(mlp, c, phi, rho, b.xin, (int)P0, b.jump, s));
    // encoder: z_l = block(down(z_{l-1})), zs_l = z_l * (w_l f(dt)); the
    // normalisation kernel also pools z_l for the next level
    for (int l = 0; l < L; ++l) {
        const Conv& k = net.enc[l];
        ConvArgs a = conv_args(k, n, Hl(l), Wl(l), l ? b.q[l - 1] : fused ? nullptr : b.xin, nullptr);
        if (!l && fused) {
            a.raw[0] = c;
            a.raw[1] = phi;
            a.raw[2] = rho;
            a.jump = jump;
        }
        a.out_f32 = b.y[l];
        GNArgs g = gn_args(h, k, n, net.P(l, 1), b.y[l], b.st[l]);
        g.stats_internal = !train;
        g.scale = b.sc[l];
        g.z_bf16 = train ? b.z[l] : nullptr;
        g.zs_bf16 = b.zs[l];
        g.pool_bf16 = l < L - 1 ? b.q[l] : nullptr;
        g.H = Hl(l);
        g.W = Wl(l);
        RCHECK(conv_gn(h, a, l ? kConvFwd : kFirst, g, !l && fused ? &mlp : nullptr, b.jump));
    }
    // bottom block
    {
        ConvArgs a = conv_args(net.mid, n, Hl(L - 1), Wl(L - 1), b.zs[L - 1], nullptr);
        a.out_f32 = b.ym;
        GNArgs g = gn_args(h, net.mid, n, net.P(L - 1, 1), b.ym, b.stm);
        g.stats_internal = !train;
        g.z_bf16 = b.am;
        RCHECK(conv_gn(h, a, kConvFwd, g));
    }
    // inference: the head convolution normalises the last decoder block's
    // output as it loads it (a_0 is not written out)
    ConvArgs head = conv_args(net.head, n, Hl(0), Wl(0), b.ad[0], nullptr);
    if (!train) {
        ConvArgs t = head;
        t.in1 = nullptr;
        t.gn_y = b.yd[0];
        t.gn_coef = b.gcoef;
        t.gn_gelu = net.dec[0].gelu;
        if (conv_gn_input_ok(t)) head = t;
    }
    for (int l = L - 2; l >= 0; --l) {
        // d_l = up(a_{l+1}); block(zs_l (+) d_l)
        const uint16_t* src = l + 1 == L - 1 ? b.am : b.ad[l + 1];
        ConvArgs u = conv_args(net.up[l + 1], n, Hl(l + 1), Wl(l + 1), src, nullptr);
        u.out_bf16 = b.d[l];
        UCHECK(conv_gemm(u, kUpFwd, s));
        ConvArgs a = conv_args(net.dec[l], n, Hl(l), Wl(l), b.zs[l], b.d[l]);
        a.out_f32 = b.yd[l];
        GNArgs g = gn_args(h, net.dec[l], n, net.P(l, 1), b.yd[l], b.std_[l]);
        g.stats_internal = !train;
        g.z_bf16 = l == 0 && head.gn_y ? nullptr : b.ad[l];
        RCHECK(conv_gn(h, a, kConvFwd, g));
    }
    // head: GN(conv(a_0)) is the rate over the leap, u' = u + dt head
    {
        ConvArgs a = head;
        a.out_f32 = b.yh;
        GNArgs g = gn_args(h, net.head, n, P0, b.yh, b.sth);
        g.res_jump = b.jump;  // the normalisation writes u + dt head directly
        g.res_in[0] = c, g.res_in[1] = phi, g.res_in[2] = rho;
        g.res_out[0] = oc, g.res_out[1] = ophi, g.res_out[2] = orho;
        RCHECK(conv_gn(h, a, kConvFwd, g));
    }
    h->last_n = train ? n : 0;
    return PF_OK;
}

int backward(unet_handle* h, const float* pc, const float* pphi, const float* prho, const float* tc,
             const float* tphi, const float* trho, double* loss_host)
{
    Net& net = h->net;
    Bufs& b = h->b;
    hipStream_t s = h->stream;
    const int L = net.L, n = h->last_n;
    const int* w = net.w;
    auto Hl = [&](int l) { return net.c.height >> l; };
    auto Wl = [&](int l) { return net.c.width >> l; };
    const long P0 = net.P(0, 1);
    UCHECK(rel_mse(pc, pphi, prho, tc, tphi, trho, b.jump, b.gout, b.lpart, b.loss, n, (int)P0, s));
    // head
    {
        GNArgs g = gn_args(h, net.head, n, P0, b.yh, b.sth);
        g.dA = b.gout;
        g.dy_bf16 = b.dyh;
        g.dgamma = grd(h, net.head.pg);
        g.dbeta = grd(h, net.head.pb);
        UCHECK(gn_backward(g, s));
        UCHECK(conv_wgrad(wgrad_args(h, n, Hl(0), Wl(0), b.dyh, net.c.out_ch, b.ad[0], w[0], nullptr, 0, 9), kConvFwd,
                          grd(h, net.head.pw), 0, s));
        ConvArgs a = dgrad_args(net.head, n, Hl(0), Wl(0), b.dyh);
        a.out_f32 = b.dad[0];
        int mode = kConvDgrad;
        if (net.head.wtk) {
            // few output channels: taps folded into K (the first layer's kernel)
            ConvArgs t = a;
            t.Wt = net.head.wtk;
            t.ldk = 64;
            t.ldo = net.head.ldo_tk;
            if (conv_wide_ok(t, kFirst)) {
                a = t;
                mode = kFirst;
            }
        }
        UCHECK(conv_gemm(a, mode, s));
    }
    // decoder, top to bottom
    for (int l = 0; l < L - 1; ++l) {
        const Conv& k = net.dec[l];
        GNArgs g = gn_args(h, k, n, net.P(l, 1), b.yd[l], b.std_[l]);
        g.dA = b.dad[l];
        g.dy_bf16 = b.dyd[l];
        g.dgamma = grd(h, k.pg);
        g.dbeta = grd(h, k.pb);
        UCHECK(gn_backward(g, s));
        UCHECK(conv_wgrad(wgrad_args(h, n, Hl(l), Wl(l), b.dyd[l], w[l], b.zs[l], w[l], b.d[l], w[l], 9), kConvFwd,
                          grd(h, k.pw), 0, s));
        ConvArgs a = dgrad_args(k, n, Hl(l), Wl(l), b.dyd[l]);
        a.out_f32 = b.dzs[l];
        a.out2_bf16 = b.dd[l];
        UCHECK(conv_gemm(a, kConvDgrad, s));
        // d_l = up(a_{l+1})
        const Conv& u = net.up[l + 1];
        const uint16_t* src = l + 1 == L - 1 ? b.am : b.ad[l + 1];
        UCHECK(conv_wgrad(wgrad_args(h, n, Hl(l + 1), Wl(l + 1), b.dd[l], 4 * w[l], src, w[l + 1], nullptr, 0, 1),
                          kUpFwd, grd(h, u.pw), 0, s));
        ConvArgs ud{};
        ud.in1 = b.dd[l];
        ud.Wt = u.wt;
        ud.out_f32 = b.dad[l + 1];
        ud.N = n;
        ud.H = Hl(l + 1);
        ud.W = Wl(l + 1);
        ud.C1 = 4 * w[l];
        ud.Nout = ud.O1 = w[l + 1];
        ud.ldk = u.ldk_t;
        ud.ldo = u.ldo_t;
        UCHECK(conv_gemm(ud, kUpDgrad, s));
    }
    // bottom block
    {
        GNArgs g = gn_args(h, net.mid, n, net.P(L - 1, 1), b.ym, b.stm);
        g.dA = b.dad[L - 1];
        g.dy_bf16 = b.dym;
        g.dgamma = grd(h, net.mid.pg);
        g.dbeta = grd(h, net.mid.pb);
        UCHECK(gn_backward(g, s));
        UCHECK(conv_wgrad(wgrad_args(h, n, Hl(L - 1), Wl(L - 1), b.dym, w[L - 1], b.zs[L - 1], w[L - 1], nullptr, 0, 9),
                          kConvFwd, grd(h, net.mid.pw), 0, s));
        ConvArgs a = dgrad_args(net.mid, n, Hl(L - 1), Wl(L - 1), b.dym);
        a.out_f32 = b.dzs[L - 1];
        UCHECK(conv_gemm(a, kConvDgrad, s));
    }
    // encoder, bottom to top
    for (int l = L - 1; l >= 0; --l) {
        const Conv& k = net.enc[l];
        GNArgs g = gn_args(h, k, n, net.P(l, 1), b.y[l], b.st[l]);
        g.scale = b.sc[l];
        if (l < L - 1) {
            // dA: the gradient of the pooling into the next level, formed
            // inside the normalisation's backward
            g.pool_z = b.z[l];
            g.pool_dq = b.dq[l];
            g.pool_tmp = b.dz[l];
            g.H = Hl(l);
            g.W = Wl(l);
        }
        g.dB = b.dzs[l];
        g.dy_bf16 = b.dye[l];
        g.dgamma = grd(h, k.pg);
        g.dbeta = grd(h, k.pb);
        g.dscale = b.ds[l];
        UCHECK(gn_backward(g, s));
        UCHECK(conv_wgrad(wgrad_args(h, n, Hl(l), Wl(l), b.dye[l], w[l], l ? b.q[l - 1] : b.xin, k.cin1, nullptr, 0, 9),
                          kConvFwd, grd(h, k.pw), 0, s));
        if (l > 0) {
            ConvArgs a = dgrad_args(k, n, Hl(l), Wl(l), b.dye[l]);
            a.out_f32 = b.dq[l - 1];
            UCHECK(conv_gemm(a, kConvDgrad, s));
        }
    }
    UCHECK(mlp_backward(mlp_args(h, n, b.jump), s));
    if (loss_host) {
        UCHECK(hipMemcpyAsync(loss_host, b.loss, sizeof(double), hipMemcpyDeviceToHost, s));
        UCHECK(hipStreamSynchronize(s));
    }
    return PF_OK;
}

}  // namespace

extern "C" {

int64_t unet_param_count(const unet_config* cfg)
{
    if (!cfg_ok(cfg)) return -1;
    try {
        return Net(*cfg).nparams;
    } catch (...) {
        return -1;
    }
}

int unet_param_entry(const unet_config* cfg, int index, unet_param_desc* out)
{
    if (!cfg_ok(cfg) || !out || index < 0) return PF_EINVAL;
    try {
        Net net(*cfg);
        if (index >= (int)net.params.size()) return PF_EINVAL;
        *out = net.params[index];
        return PF_OK;
    } catch (...) {
        return PF_EINVAL;
    }
}

size_t unet_workspace_bytes(const unet_config* cfg)
{
    if (!cfg_ok(cfg)) return 0;
    try {
        Net net(*cfg);
        Bufs b{};
        carve(net, nullptr, b);
        return b.bytes;
    } catch (...) {
        return 0;
    }
}

int unet_create(unet_handle** out, const unet_config* cfg, float* params, float* grads, void* workspace,
                size_t workspace_bytes, void* stream)
{
    if (!out) return PF_EINVAL;
    *out = nullptr;
    if (!cfg_ok(cfg) || !al(params, 4) || !al(grads, 4) || !al(workspace, 256)) return PF_EINVAL;
    unet_handle* h = nullptr;
    try {
        h = new unet_handle(*cfg);
    } catch (...) {
        return PF_EINVAL;
    }
    carve(h->net, (char*)workspace, h->b);
    if (workspace_bytes < h->b.bytes) {
        delete h;
        return PF_EINVAL;
    }
    h->params = params;
    h->grads = grads;
    h->stream = (hipStream_t)stream;
    // no memo entry is valid yet (generation 0 is never used)
    if (fill_f32((float*)h->b.mlpc, (size_t)cfg->max_batch * h->net.L * 2, 0.f, h->stream) != hipSuccess) {
        delete h;
        return PF_EDEVICE;
    }
    const int rc = prepare_all(h);
    if (rc != PF_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return PF_OK;
}

int unet_prepare(unet_handle* h)
{
    if (!h) return PF_EINVAL;
    return prepare_all(h);
}

int unet_forward(unet_handle* h, int n, const float* jump, const float* c, const float* phi, const float* rho,
                 float* oc, float* ophi, float* orho)
{
    if (!h || n <= 0 || n > h->net.c.max_batch) return PF_EINVAL;
    if (!al(jump, 4) || !al(c, 4) || !al(phi, 4) || !al(rho, 4) || !al(oc, 4) || !al(ophi, 4) || !al(orho, 4))
        return PF_EINVAL;
    return forward(h, n, jump, c, phi, rho, oc, ophi, orho, true);
}

int unet_forward_infer(unet_handle* h, int n, const float* jump, const float* c, const float* phi, const float* rho,
                       float* oc, float* ophi, float* orho)
{
    if (!h || n <= 0 || n > h->net.c.max_batch) return PF_EINVAL;
    if (!al(jump, 4) || !al(c, 4) || !al(phi, 4) || !al(rho, 4) || !al(oc, 4) || !al(ophi, 4) || !al(orho, 4))
        return PF_EINVAL;
    return forward(h, n, jump, c, phi, rho, oc, ophi, orho, false);
}

int unet_backward(unet_handle* h, const float* pc, const float* pphi, const float* prho, const float* tc,
                  const float* tphi, const float* trho, double* loss)
{
    if (!h || h->last_n <= 0) return PF_EINVAL;
    if (!al(pc, 4) || !al(pphi, 4) || !al(prho, 4) || !al(tc, 4) || !al(tphi, 4) || !al(trho, 4)) return PF_EINVAL;
    return backward(h, pc, pphi, prho, tc, tphi, trho, loss);
}

int unet_adam(unet_handle* h, float* m, float* v, int64_t t, float lr, float beta1, float beta2, float eps)
{
    if (!h || !al(m, 4) || !al(v, 4) || t < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
        !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return PF_EINVAL;
    const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)t));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)t));
    UCHECK(adam_update(h->params, h->grads, m, v, (size_t)h->net.nparams, lr, beta1, beta2, eps, bc1, bc2, h->stream));
    return prepare_all(h);
}

void unet_destroy(unet_handle* h) { delete h; }

}  // extern "C"

// ------------------------------------------------------------ single ops
namespace {

struct OpWs {
    char* p;
    size_t left;
    bool ok = true;
    template <class T>
    T* take(size_t count)
    {
        const size_t b = r256(count * sizeof(T));
        if (b > left) {
            ok = false;
            return nullptr;
        }
        T* r = (T*)p;
        p += b;
        left -= b;
        return r;
    }
};

bool dims_ok(int n, int H, int W) { return n > 0 && H > 0 && W > 0 && (long)n * H * W <= (1L << 30); }

}  // namespace

extern "C" {

size_t unet_op_workspace_bytes(int n, int H, int W, int Cmax)
{
    if (!dims_ok(n, H, W) || Cmax <= 0) return 0;
    const size_t C = (size_t)Cmax;
    const size_t wconv = 9 * r128(C) * r32(C), wup = r128(4 * C) * r32(C) + r128(C) * r32(4 * C);
    const size_t wbytes = r256(2 * std::max(wconv, wup)) + r256(2 * 9 * r128(C) * r32(C));
    const size_t part = (size_t)4194304 + 9 * C * 4 * C;
    const size_t P = (size_t)H * W;
    const size_t csum = gn_csum_floats(n, (int)std::min(P, (size_t)1 << 30), Cmax);
    return wbytes + r256(4 * part) + r256(4 * csum) + r256(8 * (size_t)n * 5 * C) + 4096;
}

size_t unet_conv3x3_prep_bytes(int C1, int C2, int Cout)
{
    if (C1 <= 0 || C2 < 0 || Cout <= 0) return 0;
    return r256(2 * 9 * r128(Cout) * r32(C1 + C2));
}

int unet_conv3x3_prepare(const float* w, int C1, int C2, int Cout, void* wprep, size_t bytes, void* stream)
{
    if (C1 <= 0 || C2 < 0 || Cout <= 0 || !al(w, 4) || !al(wprep, 256)) return PF_EINVAL;
    if (bytes < unet_conv3x3_prep_bytes(C1, C2, Cout)) return PF_EINVAL;
    const int K = C1 + C2;
    UCHECK(weight_prep(w, 9, Cout, K, (uint16_t*)wprep, (int)r128(Cout), (int)r32(K), nullptr, 0, 0,
                       (hipStream_t)stream));
    return PF_OK;
}

int unet_conv3x3_fwd_prepared(int n, int H, int W, const uint16_t* x1, int C1, const uint16_t* x2, int C2,
                              const void* wprep, int Cout, float* y, void* stream)
{
    if (!dims_ok(n, H, W) || C1 <= 0 || C2 < 0 || Cout <= 0 || !al(x1, 8) || !al(wprep, 256) || !al(y, 4))
        return PF_EINVAL;
    if (C2 > 0 && (!al(x2, 8) || C1 % 4)) return PF_EINVAL;
    const int K = C1 + C2;
    ConvArgs a{};
    a.in1 = x1;
    a.in2 = C2 ? x2 : nullptr;
    a.Wt = (const uint16_t*)wprep;
    a.out_f32 = y;
    a.N = n;
    a.H = H;
    a.W = W;
    a.C1 = C1;
    a.C2 = C2;
    a.Nout = a.O1 = Cout;
    a.ldk = (int)r32(K);
    a.ldo = (int)r128(Cout);
    UCHECK(conv_gemm(a, kConvFwd, (hipStream_t)stream));
    return PF_OK;
}

int unet_conv3x3_fwd(int n, int H, int W, const uint16_t* x1, int C1, const uint16_t* x2, int C2, const float* w,
                     int Cout, float* y, void* workspace, size_t workspace_bytes, void* stream)
{
    if (!dims_ok(n, H, W) || C1 <= 0 || C2 < 0 || Cout <= 0 || !al(x1, 8) || !al(w, 4) || !al(y, 4) ||
        !al(workspace, 256))
        return PF_EINVAL;
    if (C2 > 0 && (!al(x2, 8) || C1 % 4)) return PF_EINVAL;
    const size_t wb = unet_conv3x3_prep_bytes(C1, C2, Cout);
    if (workspace_bytes < wb) return PF_EINVAL;
    const int rc = unet_conv3x3_prepare(w, C1, C2, Cout, workspace, wb, stream);
    if (rc != PF_OK) return rc;
    return unet_conv3x3_fwd_prepared(n, H, W, x1, C1, x2, C2, workspace, Cout, y, stream);
}

int unet_conv3x3_dgrad(int n, int H, int W, const uint16_t* dy, int Cout, const float* w, int C1, int C2, float* dx1,
                       float* dx2, void* workspace, size_t workspace_bytes, void* stream)
{
    if (!dims_ok(n, H, W) || C1 <= 0 || C2 < 0 || Cout <= 0 || !al(dy, 8) || !al(w, 4) || !al(dx1, 4) ||
        !al(workspace, 256))
        return PF_EINVAL;
    if (C2 > 0 && !al(dx2, 4)) return PF_EINVAL;
    const int K = C1 + C2;
    OpWs ws{(char*)workspace, workspace_bytes};
    uint16_t* wt = ws.take<uint16_t>(9 * r128(K) * r32(Cout));
    if (!ws.ok) return PF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    UCHECK(weight_prep(w, 9, Cout, K, nullptr, 0, 0, wt, (int)r128(K), (int)r32(Cout), s));
    ConvArgs a{};
    a.in1 = dy;
    a.Wt = wt;
    a.out_f32 = dx1;
    a.out2_f32 = C2 ? dx2 : nullptr;
    a.N = n;
    a.H = H;
    a.W = W;
    a.C1 = Cout;
    a.Nout = K;
    a.O1 = C1;
    a.ldk = (int)r32(Cout);
    a.ldo = (int)r128(K);
    if (Cout <= 4 && C2 == 0) {
        // few gradient channels: taps folded into K, as in the network's head
        ConvArgs t = a;
        uint16_t* wk = ws.take<uint16_t>(r128(K) * 64);
        t.Wt = wk;
        t.ldk = 64;
        t.ldo = (int)r128(K);
        if (ws.ok && conv_wide_ok(t, kFirst)) {
            PrepItem p{};
            p.kind = kPrepFirstGrad;
            p.W = w;
            p.taps = 9;
            p.R = Cout;
            p.Kc = K;
            p.tr = wk;
            p.ldo_t = t.ldo;
            UCHECK(weight_prep_batch(&p, 1, s));
            UCHECK(conv_gemm(t, kFirst, s));
            return PF_OK;
        }
    }
    UCHECK(conv_gemm(a, kConvDgrad, s));
    return PF_OK;
}

int unet_conv3x3_wgrad(int n, int H, int W, const uint16_t* dy, int Cout, const uint16_t* x1, int C1,
                       const uint16_t* x2, int C2, float* dw, void* workspace, size_t workspace_bytes, void* stream)
{
    if (!dims_ok(n, H, W) || C1 <= 0 || C2 < 0 || Cout <= 0 || !al(dy, 2) || !al(x1, 2) || !al(dw, 4) ||
        !al(workspace, 256))
        return PF_EINVAL;
    if (C2 > 0 && !al(x2, 2)) return PF_EINVAL;
    const long P = (long)n * H * W;
    OpWs ws{(char*)workspace, workspace_bytes};
    WgradArgs a{};
    a.dy = dy;
    a.x1 = x1;
    a.x2 = C2 ? x2 : nullptr;
    a.N = n;
    a.H = H;
    a.W = W;
    a.C1 = C1;
    a.C2 = C2;
    a.Nout = Cout;
    a.chunk = wgrad_chunk(P, 9, Cout, C1, C2);
    const size_t pf = wgrad_floats(P, 9, Cout, C1, C2);
    a.partial = ws.take<float>(pf);
    a.partial_cap = pf;
    if (!ws.ok) return PF_EINVAL;
    UCHECK(conv_wgrad(a, kConvFwd, dw, 0, (hipStream_t)stream));
    return PF_OK;
}

int unet_up_fwd(int n, int H, int W, const uint16_t* x, int Cin, const float* w, int Cout, float* y, void* workspace,
                size_t workspace_bytes, void* stream)
{
    if (!dims_ok(n, 2 * H, 2 * W) || Cin <= 0 || Cout <= 0 || !al(x, 8) || !al(w, 4) || !al(y, 4) ||
        !al(workspace, 256))
        return PF_EINVAL;
    OpWs ws{(char*)workspace, workspace_bytes};
    uint16_t* wf = ws.take<uint16_t>(r128(4 * Cout) * r32(Cin));
    if (!ws.ok) return PF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    UCHECK(weight_prep(w, 1, 4 * Cout, Cin, wf, (int)r128(4 * Cout), (int)r32(Cin), nullptr, 0, 0, s));
    ConvArgs a{};
    a.in1 = x;
    a.Wt = wf;
    a.out_f32 = y;
    a.N = n;
    a.H = H;
    a.W = W;
    a.C1 = Cin;
    a.Nout = a.O1 = 4 * Cout;
    a.ldk = (int)r32(Cin);
    a.ldo = (int)r128(4 * Cout);
    UCHECK(conv_gemm(a, kUpFwd, s));
    return PF_OK;
}

int unet_up_dgrad(int n, int H, int W, const uint16_t* dy, int Cout, const float* w, int Cin, float* dx,
                  void* workspace, size_t workspace_bytes, void* stream)
{
    if (!dims_ok(n, 2 * H, 2 * W) || Cin <= 0 || Cout <= 0 || Cout % 4 || !al(dy, 8) || !al(w, 4) || !al(dx, 4) ||
        !al(workspace, 256))
        return PF_EINVAL;
    OpWs ws{(char*)workspace, workspace_bytes};
    uint16_t* wt = ws.take<uint16_t>(r128(Cin) * r32(4 * Cout));
    if (!ws.ok) return PF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    UCHECK(weight_prep(w, 1, 4 * Cout, Cin, nullptr, 0, 0, wt, (int)r128(Cin), (int)r32(4 * Cout), s));
    ConvArgs a{};
    a.in1 = dy;
    a.Wt = wt;
    a.out_f32 = dx;
    a.N = n;
    a.H = H;
    a.W = W;
    a.C1 = 4 * Cout;
    a.Nout = a.O1 = Cin;
    a.ldk = (int)r32(4 * Cout);
    a.ldo = (int)r128(Cin);
    UCHECK(conv_gemm(a, kUpDgrad, s));
    return PF_OK;
}

int unet_up_wgrad(int n, int H, int W, const uint16_t* dy, int Cout, const uint16_t* x, int Cin, float* dw,
                  void* workspace, size_t workspace_bytes, void* stream)
{
    if (!dims_ok(n, 2 * H, 2 * W) || Cin <= 0 || Cout <= 0 || !al(dy, 2) || !al(x, 2) || !al(dw, 4) ||
        !al(workspace, 256))
        return PF_EINVAL;
    const long P = (long)n * H * W;
    OpWs ws{(char*)workspace, workspace_bytes};
    WgradArgs a{};
    a.dy = dy;
    a.x1 = x;
    a.N = n;
    a.H = H;
    a.W = W;
    a.C1 = Cin;
    a.Nout = 4 * Cout;
    a.chunk = wgrad_chunk(P, 1, 4 * Cout, Cin, 0);
    a.partial = ws.take<float>(wgrad_floats(P, 1, 4 * Cout, Cin, 0));
    if (!ws.ok) return PF_EINVAL;
    UCHECK(conv_wgrad(a, kUpFwd, dw, 0, (hipStream_t)stream));
    return PF_OK;
}

static bool gn_dims_ok(int n, int P, int C, int G)
{
    return n > 0 && P > 0 && C > 0 && C <= 256 && G > 0 && C % G == 0 && (long)n * P <= (1L << 30);
}

int unet_groupnorm_fwd(int n, int P, int C, int G, float eps, int gelu, const float* y, const float* gamma,
                       const float* beta, const float* scale, float* z, float* zs, float* stats, void* workspace,
                       size_t workspace_bytes, void* stream)
{
    if (!gn_dims_ok(n, P, C, G) || !(eps > 0.f) || !al(y, 4) || !al(gamma, 4) || !al(beta, 4) || !al(z, 4) ||
        !al(stats, 4) || !al(workspace, 256))
        return PF_EINVAL;
    if ((zs && !scale) || (scale && !al(scale, 4))) return PF_EINVAL;
    OpWs ws{(char*)workspace, workspace_bytes};
    GNArgs g{};
    g.csum = ws.take<float>(gn_csum_floats(n, P, C));
    g.cacc = ws.take<double>((size_t)n * (3 * C + 2 * G));
    if (!ws.ok) return PF_EINVAL;
    g.y = y;
    g.gamma = gamma;
    g.beta = beta;
    g.scale = scale;
    g.stats = stats;
    g.z_f32 = z;
    g.zs_f32 = zs;
    g.N = n;
    g.P = P;
    g.C = C;
    g.G = G;
    g.gelu = gelu ? 1 : 0;
    g.eps = eps;
    UCHECK(gn_forward(g, (hipStream_t)stream));
    return PF_OK;
}

int unet_groupnorm_bwd(int n, int P, int C, int G, float eps, int gelu, const float* y, const float* gamma,
                       const float* beta, const float* scale, const float* stats, const float* dA, const float* dB,
                       float* dy, float* dgamma, float* dbeta, float* dscale, void* workspace,
                       size_t workspace_bytes, void* stream)
{
    if (!gn_dims_ok(n, P, C, G) || !(eps > 0.f) || !al(y, 4) || !al(gamma, 4) || !al(beta, 4) || !al(stats, 4) ||
        !al(dy, 4) || !al(dgamma, 4) || !al(dbeta, 4) || !al(workspace, 256))
        return PF_EINVAL;
    if (!dA && !dB) return PF_EINVAL;
    if (dscale && (!scale || !dB)) return PF_EINVAL;
    OpWs ws{(char*)workspace, workspace_bytes};
    GNArgs g{};
    g.csum = ws.take<float>(gn_csum_floats(n, P, C));
    g.cacc = ws.take<double>((size_t)n * (3 * C + 2 * G));
    if (!ws.ok) return PF_EINVAL;
    g.y = y;
    g.gamma = gamma;
    g.beta = beta;
    g.scale = scale;
    g.stats = (float*)stats;
    g.dA = dA;
    g.dB = dB;
    g.dy_f32 = dy;
    g.dgamma = dgamma;
    g.dbeta = dbeta;
    g.dscale = dscale;
    g.N = n;
    g.P = P;
    g.C = C;
    g.G = G;
    g.gelu = gelu ? 1 : 0;
    g.eps = eps;
    UCHECK(gn_backward(g, (hipStream_t)stream));
    return PF_OK;
}

int unet_maxpool_fwd(int n, int H, int W, int C, const uint16_t* x, uint16_t* y, void* stream)
{
    if (!dims_ok(n, H, W) || H % 2 || W % 2 || C <= 0 || !al(x, 2) || !al(y, 2)) return PF_EINVAL;
    UCHECK(maxpool_fwd(x, y, n, H, W, C, (hipStream_t)stream));
    return PF_OK;
}

int unet_maxpool_bwd(int n, int H, int W, int C, const uint16_t* x, const float* dy, float* dx, void* stream)
{
    if (!dims_ok(n, H, W) || H % 2 || W % 2 || C <= 0 || !al(x, 2) || !al(dy, 4) || !al(dx, 4)) return PF_EINVAL;
    UCHECK(maxpool_bwd(x, dy, dx, n, H, W, C, (hipStream_t)stream));
    return PF_OK;
}

}  // extern "C"
