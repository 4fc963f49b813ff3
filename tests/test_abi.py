"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/pf.h declares, its host-only entry points agree with
the oracle, and argument errors are reported before anything is enqueued."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2312_05410_amd import _lib
from paper_2312_05410_amd.inputs import PFParams, uniform01

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "pf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_params_struct_layout():
    # int32 x 12, uint64 seed at 48, 21 doubles, 2 pointers
    assert _lib.PFParamsC.seed.offset == 48
    assert _lib.PFParamsC.h.offset == 56
    assert _lib.PFParamsC.v0_per.offset == 56 + 21 * 8
    assert _lib.PFParamsC.integrator.offset == 44
    assert _lib.PFParamsC.interface_noise.offset == 56 + 21 * 8 + 16
    assert _lib.PFParamsC.lane_cols.offset == 56 + 21 * 8 + 24
    assert _lib.PFParamsC.fused_kernel.offset == 56 + 21 * 8 + 28
    assert ctypes.sizeof(_lib.PFParamsC) == 56 + 21 * 8 + 32


def test_strerror():
    L = _lib.load()
    for code in (0, -1, -2, -3, -4, -5, -6, 7):
        assert L.pf_strerror(code)


@pytest.mark.parametrize("seed", range(6))
def test_dt_limit_matches_oracle(seed):
    """Random parameter sets exercise every field the stability rule reads
    (also a check that the struct fields line up)."""
    u = uniform01(100 + seed, np.arange(16))
    p = PFParams(h=0.5 + u[0], W_c=0.2 + 2 * u[1], W_phi=0.2 + 2 * u[2], kappa_c=0.1 + 2 * u[3],
                 kappa_phi=0.1 + 3 * u[4], MA_bulk=2 * u[5], MB_bulk=2 * u[6], MA_surf=6 * u[7],
                 MB_surf=6 * u[8], M_phi=0.1 + u[9], M_scale=0.5 + u[10], D_rho=0.1 + u[11],
                 v0=3 * u[12] + (5 if seed % 2 else 0), flux_on=seed != 4)
    assert _lib.dt_limit(p) == pytest.approx(oracle.dt_limit(p), rel=1e-15)


def test_dt_limit_batch_uses_fastest_realisation():
    p = PFParams(batch=3, v0_per=np.array([0.5, 30.0, 1.0]))
    assert _lib.dt_limit(p) == pytest.approx(2 * p.D_rho / 900.0, rel=1e-15)


def test_workspace_bytes():
    p = PFParams(nx=100, ny=60, batch=2, precision="f32")
    n = _lib.workspace_bytes(p)
    assert n >= 3 * 2 * 100 * 60 * 4 + 2 * 100 * 8
    assert n % 256 == 0
    assert _lib.workspace_bytes(p.replace(precision="f64")) > n


def _ws(p, **kw):
    s, keep = _lib.to_c(p, **kw)
    return _lib.load().pf_workspace_bytes(ctypes.byref(s))


def test_resident_stepper_shapes_and_workspace():
    """The resident stepper's shape rules are checked before anything runs;
    its rim buffers (2 x tiles x 3 x (256 + 4 TY) 8-byte words) and its
    256-byte control block are in the workspace exactly when it may run."""
    base = PFParams(nx=128, ny=64, precision="f32")
    n0 = _ws(base)                                   # 8192 cells: no resident stepper by default
    assert _ws(base, fused_kernel=3) - n0 == 2 * 4 * 3 * (256 + 4 * 32) * 8 + 256          # TY 32: 2 x 2 tiles
    assert _ws(base, fused_kernel=3, tile_rows=8) - n0 == 2 * 16 * 3 * (256 + 4 * 8) * 8 + 256
    assert _ws(base, fused_kernel=3, temporal_block=1) == _ws(base, fused_kernel=3)
    big = PFParams(nx=512, ny=512, precision="f32")  # 2^18 cells: the default
    assert _ws(big) - _ws(big, temporal_block=2) == 2 * 128 * 3 * (256 + 4 * 32) * 8 + 256
    assert _ws(big, tile_rows=8) == _ws(big, temporal_block=2)   # a chunk height asked for: no resident
    assert _ws(base.replace(integrator="midpoint"), fused_kernel=3) == _ws(base, fused_kernel=3)
    assert _ws(base.replace(interface_noise=0.1), fused_kernel=3) == _ws(base, fused_kernel=3)
    assert _ws(big.replace(interface_noise=0.1)) == _ws(big)          # draws in the resident stepper too
    for bad in (dict(nx=100), dict(precision="f64"), dict(ny=60),
                dict(nx=2048, ny=2048)):
        assert _ws(base.replace(**bad), fused_kernel=3) == 0, bad
    assert _ws(base, fused_kernel=3, temporal_block=2) == 0
    assert _ws(base, fused_kernel=3, tile_rows=4) == 0
    assert _ws(base, fused_kernel=4) == 0


def _init(p, ptrs=(4096, 8192, 12288), ws=1 << 20, wsize=None, **kw):
    L = _lib.load()
    s, keep = _lib.to_c(p, **kw)
    h = ctypes.c_void_p()
    n = wsize if wsize is not None else L.pf_workspace_bytes(ctypes.byref(s))
    return L.pf_init(ctypes.byref(h), ctypes.byref(s), ptrs[0], ptrs[1], ptrs[2], ws, n, None), h


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-3), dict(batch=0), dict(precision="f16"), dict(h=0.0), dict(sigma_surf=0.0),
    dict(MA_bulk=-1.0), dict(D_rho=-0.1), dict(dt=0.0, dt_factor=0.0), dict(W_c=float("nan")),
    dict(v0=float("inf")),
])
def test_init_rejects_bad_params(bad):
    if bad.get("precision") == "f16":
        with pytest.raises(KeyError):
            _lib.to_c(PFParams(**bad))
        return
    rc, h = _init(PFParams(**bad))
    assert rc == _lib.PF_EINVAL and not h.value


def test_init_rejects_bad_pointers_and_workspace():
    p = PFParams(nx=16, ny=16)
    assert _init(p, ptrs=(0, 8192, 12288))[0] == _lib.PF_EINVAL
    assert _init(p, ptrs=(4096 + 4, 8192, 12288))[0] == _lib.PF_EINVAL   # misaligned field
    assert _init(p, ws=0)[0] == _lib.PF_EINVAL
    assert _init(p, ws=4096 + 64)[0] == _lib.PF_EINVAL                   # workspace not 256-aligned
    assert _init(p, wsize=1024)[0] == _lib.PF_EINVAL                      # workspace too small
    assert _init(p, temporal_block=5)[0] == _lib.PF_EINVAL
    assert _init(p, tile_rows=12)[0] == _lib.PF_EINVAL
    assert _init(p, lane_cols=3)[0] == _lib.PF_EINVAL
    assert _init(p, lane_cols=-1)[0] == _lib.PF_EINVAL
    assert _init(p, fused_kernel=3)[0] == _lib.PF_EINVAL
    assert _init(p, fused_kernel=2, temporal_block=3)[0] == _lib.PF_EINVAL
    assert _init(p.replace(precision="f64"), temporal_block=3)[0] == _lib.PF_EINVAL
    L = _lib.load()
    assert L.pf_step_n(None, 3) == _lib.PF_EINVAL
    assert L.pf_mass(None, None) == _lib.PF_EINVAL


def test_init_rejects_unstable_dt():
    p = PFParams(nx=16, ny=16)
    lim = oracle.dt_limit(p)
    rc, _ = _init(p.replace(dt=1.01 * lim))
    assert rc == _lib.PF_EUNSTABLE


def test_product_path_has_no_oracle_import():
    """The package never imports the oracle (test infrastructure only)."""
    pkg = os.path.join(ROOT, "paper_2312_05410_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "pf_oracle" not in text, f


# ------------------------------------------------------------------ U-Net
def test_unet_library_exports_every_declared_symbol():
    from paper_2312_05410_amd import unet

    text = open(os.path.join(ROOT, "include", "unet.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(unet_[a-z0-9_]+)\s*\(", text)))
    L = unet.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(unet.UNET_EXPORTS)


def test_unet_struct_layouts():
    from paper_2312_05410_amd import unet

    assert ctypes.sizeof(unet.UNetConfigC) == 12 * 4
    assert unet.ParamDescC.offset.offset == 32 and ctypes.sizeof(unet.ParamDescC) == 32 + 8 + 8 + 4 + 16 + 4


def test_unet_param_layout_and_validation():
    from paper_2312_05410_amd import unet

    cfg = unet.UNetConfig()
    e = unet.param_entries(cfg)
    names = [x[0] for x in e]
    assert names[:3] == ["enc0.w", "enc0.gamma", "enc0.beta"] and names[-1] == "film3.w"
    d = dict((x[0], x[2]) for x in e)
    assert d["enc0.w"] == (9, 32, 4) and d["mid.w"] == (9, 256, 256) and d["up3.w"] == (4, 128, 256)
    assert d["dec0.w"] == (9, 32, 64) and d["head.w"] == (9, 3, 32) and d["film2.w"] == (128, 128)
    offs = [x[1] for x in e]
    assert offs == sorted(offs) and offs[0] == 0
    L = unet.lib()
    for bad in (dict(in_ch=3), dict(out_ch=4), dict(levels=1), dict(height=100), dict(base=6), dict(groups=5),
                dict(mlp_hidden=300), dict(head_groups=2), dict(gn_eps=0.0), dict(max_batch=0), dict(base=128),
                dict(base=4), dict(base=12)):
        c = unet.UNetConfig(**{**cfg.__dict__, **bad})
        assert L.unet_param_count(ctypes.byref(c.c())) == -1, bad
        assert L.unet_workspace_bytes(ctypes.byref(c.c())) == 0, bad
    h = ctypes.c_void_p()
    rc = L.unet_create(ctypes.byref(h), ctypes.byref(cfg.c()), None, None, None, 0, None)
    assert rc == _lib.PF_EINVAL and not h.value


def test_unet_ops_reject_bad_arguments():
    """Shape and pointer errors are caught before any device work."""
    from paper_2312_05410_amd import unet

    L = unet.lib()
    fake = 4096  # aligned non-null value: never dereferenced, every call below fails validation first
    assert L.unet_conv3x3_fwd(0, 4, 4, fake, 4, None, 0, fake, 8, fake, fake, 1 << 20, None) == _lib.PF_EINVAL
    assert L.unet_conv3x3_fwd(1, 4, 4, fake, 6, fake, 4, fake, 8, fake, fake, 1 << 20, None) == _lib.PF_EINVAL
    assert L.unet_conv3x3_fwd(1, 4, 4, fake + 2, 4, None, 0, fake, 8, fake, fake, 1 << 20, None) == _lib.PF_EINVAL
    assert L.unet_conv3x3_fwd(1, 4, 4, fake, 4, None, 0, fake, 8, fake, fake, 16, None) == _lib.PF_EINVAL
    assert L.unet_up_dgrad(1, 4, 4, fake, 6, fake, 8, fake, fake, 1 << 20, None) == _lib.PF_EINVAL
    assert L.unet_groupnorm_fwd(1, 16, 10, 3, 1e-5, 1, fake, fake, fake, None, fake, None, fake, fake, 1 << 20,
                                None) == _lib.PF_EINVAL
    assert L.unet_groupnorm_fwd(1, 16, 300, 3, 1e-5, 1, fake, fake, fake, None, fake, None, fake, fake, 1 << 20,
                                None) == _lib.PF_EINVAL
    assert L.unet_maxpool_fwd(1, 5, 4, 8, fake, fake, None) == _lib.PF_EINVAL


def test_c_struct_layouts_match_the_bindings(tmp_path):
    """Compile a probe against include/*.h with the host C compiler and
    compare every field offset and struct size with the ctypes mirrors."""
    import subprocess

    from paper_2312_05410_amd import unet

    probes = [("pf_params", "pf.h", _lib.PFParamsC), ("unet_config", "unet.h", unet.UNetConfigC),
              ("unet_param_desc", "unet.h", unet.ParamDescC)]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "pf.h"', '#include "unet.h"', "int main(void) {"]
    for cname, _, cls in probes:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _t in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        name, field, val = line.split()
        got[(name, field)] = int(val)
    for cname, _, cls in probes:
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _t in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


@pytest.mark.parametrize("bad", [dict(integrator=2), dict(interface_noise=-0.1), dict(interface_noise=2.0)])
def test_variant_params_validated(bad):
    L = _lib.load()
    s, keep = _lib.to_c(PFParams(nx=16, ny=16))
    for k, v in bad.items():
        setattr(s, k, v)
    assert L.pf_workspace_bytes(ctypes.byref(s)) == 0


def test_variants_need_the_single_step_kernel():
    L = _lib.load()
    s, keep = _lib.to_c(PFParams(nx=16, ny=16, integrator="midpoint"), temporal_block=2)
    assert L.pf_workspace_bytes(ctypes.byref(s)) == 0
    s, keep = _lib.to_c(PFParams(nx=16, ny=16, interface_noise=0.1), temporal_block=3)
    assert L.pf_workspace_bytes(ctypes.byref(s)) == 0
    s, keep = _lib.to_c(PFParams(nx=16, ny=16, integrator="midpoint", interface_noise=0.1), temporal_block=1)
    assert L.pf_workspace_bytes(ctypes.byref(s)) > 0


def test_adjoint_refuses_midpoint_and_interface_draws():
    """The adjoint is the transpose of the explicit Euler step without
    interface draws: the workspace query refuses the other model variants
    (0 bytes), and the autograd wrapper raises before running anything."""
    L = _lib.load()
    base = PFParams(nx=64, ny=32, precision="f32", dt=1e-4)
    for p, ok in ((base, True), (base.replace(integrator="midpoint"), False),
                  (base.replace(interface_noise=0.1), False)):
        s, keep = _lib.to_c(p)
        n = L.pf_adjoint_workspace_bytes(ctypes.byref(s))
        assert (n > 0) == ok, (p.integrator, p.interface_noise)
    from paper_2312_05410_amd import adjoint

    torch = pytest.importorskip("torch")
    u0 = [torch.zeros((1, 32, 64), dtype=torch.float32) for _ in range(3)]
    for p in (base.replace(integrator="midpoint"), base.replace(interface_noise=0.1)):
        with pytest.raises(ValueError):
            adjoint.final_state(1.0, 0.5, p, u0, 4, every=2)
