"""Pins of the CPU FP64 oracle against what the mathematics fixes.

The paper prints no worked example of the phase-field step, so parity with
the paper itself is unpinned; these tests tie the oracle to closed forms
(Fourier and cosine symbols of the discrete operators, linearised growth
factors), invariants of the model's conservation / gradient-flow form
(mass, the phi+rho inflow budget, energy decay), an independent dense
assembly on tiny grids, the energy-gradient identity mu = dF/du, and the
published SplitMix64 outputs.  Each is chosen so that a dropped term, a
wrong sign or index, or a transposed axis in the oracle fails one of them.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from paper_2312_05410_amd.inputs import PFParams, initial_state, random_state, splitmix64, uniform01
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lam_h(kx, ky, h=1.0):
    """Symbol of minus the 5-point Laplacian on a periodic grid."""
    return 4.0 / h**2 * (np.sin(kx * h / 2) ** 2 + np.sin(ky * h / 2) ** 2)


# ------------------------------------------------------------------ RNG / IC

def test_splitmix64_published_vectors():
    lines = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) if not l.startswith("#")]
    seed = int(lines[0][1])
    want = [int(l[0]) for l in lines[1:]]
    assert [oracle.splitmix64(seed, n) for n in range(len(want))] == want
    assert oracle.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert list(splitmix64(seed, np.arange(len(want)))) == want


def test_seeded_init_matches_input_generator():
    p = PFParams(nx=40, ny=24, batch=3, seed=7, c0_per=np.array([0.31, 0.5, 0.69]))
    c, phi, rho = oracle.init(p)
    c2, phi2, rho2 = initial_state(p)
    assert np.array_equal(c, c2)
    np.testing.assert_allclose(phi, phi2, rtol=0, atol=2e-16)
    np.testing.assert_allclose(rho, rho2, rtol=0, atol=2e-16)
    # noise amplitude and mean as configured
    for b in range(3):
        d = c[b] - p.c0_per[b]
        assert np.all(np.abs(d) <= p.c_noise) and abs(d.mean()) < 2e-3
    # realisation b equals a single run with seed + b
    cb, _, _ = oracle.init(p.replace(batch=1, seed=9, c0_per=None, c0=0.69))
    assert np.array_equal(cb[0], c[2])


# ------------------------------------------------------- discrete operators

@pytest.mark.parametrize("kx,ky", [(1, 0), (0, 3), (5, 2), (16, 7)])
def test_laplacian_fourier_symbol(kx, ky):
    """Periodic: with W = 0, mu_c = -kappa_c Lap c and Lap cos(k.x) = -lam_h cos(k.x)."""
    nx, ny = 32, 16
    p = PFParams(nx=nx, ny=ny, bc_mode="periodic", W_c=0.0, W_phi=0.0, kappa_c=1.0, kappa_phi=1.0, h=0.7)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny))
    Kx, Ky = 2 * np.pi * kx / (nx * p.h), 2 * np.pi * ky / (ny * p.h)
    u = np.cos(Kx * i * p.h + Ky * j * p.h)
    mc, mp, _ = oracle.potentials(p, u, u)
    lam = lam_h(Kx, Ky, p.h)
    np.testing.assert_allclose(mc, lam * u, rtol=0, atol=1e-13 * max(lam, 1))
    np.testing.assert_allclose(mp, lam * u, rtol=0, atol=1e-13 * max(lam, 1))


@pytest.mark.parametrize("ky", [1, 2, 7])
def test_laplacian_mirror_cosine_modes(ky):
    """PVD mirror ghosts: cos(pi k (j+1/2)/ny) are eigenvectors of the
    zero-flux 5-point Laplacian with eigenvalue -(4/h^2) sin^2(pi k / 2 ny)."""
    nx, ny = 8, 12
    p = PFParams(nx=nx, ny=ny, W_c=0.0, W_phi=0.0, kappa_c=1.0, kappa_phi=1.0)
    j = np.arange(ny)[:, None] * np.ones((1, nx))
    u = np.cos(np.pi * ky * (j + 0.5) / ny)
    mc, _, _ = oracle.potentials(p, u, u)
    lam = 4 * np.sin(np.pi * ky / (2 * ny)) ** 2
    np.testing.assert_allclose(mc, lam * u, rtol=0, atol=1e-14)


def test_laplacian_exact_on_quadratic_interior():
    nx, ny = 8, 10
    p = PFParams(nx=nx, ny=ny, W_c=0.0, W_phi=0.0, kappa_c=1.0, kappa_phi=1.0, h=0.5)
    y = (np.arange(ny)[:, None] + 0.5) * p.h * np.ones((1, nx))
    mc, _, _ = oracle.potentials(p, y**2, y**2)
    # interior rows: Lap y^2 = 2 exactly; mu = -Lap
    np.testing.assert_allclose(mc[1:-1], -2.0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("bc", ["pvd", "periodic"])
def test_mu_is_energy_gradient(bc):
    """h^2 mu_c = dF_h/dc and h^2 mu_phi = dF_h/dphi, cell by cell (central FD)."""
    nx, ny = 8, 8
    p = PFParams(nx=nx, ny=ny, bc_mode=bc, h=0.8, W_c=1.3, W_phi=0.9, kappa_c=0.7, kappa_phi=1.9)
    c, phi, _ = random_state(3, 1, ny, nx)
    c, phi = c[0], phi[0]
    mc, mp, _ = oracle.potentials(p, c, phi)
    P1 = p.replace(batch=1)

    def F(cc, pp):
        return oracle.State(P1, cc[None], pp[None], np.zeros((1, ny, nx)), dt=1.0).energy()[0]

    eps = 1e-5
    gc = np.zeros_like(c)
    gp = np.zeros_like(c)
    for j in range(ny):
        for i in range(nx):
            d = np.zeros_like(c)
            d[j, i] = eps
            gc[j, i] = (F(c + d, phi) - F(c - d, phi)) / (2 * eps)
            gp[j, i] = (F(c, phi + d) - F(c, phi - d)) / (2 * eps)
    h2 = p.h**2
    np.testing.assert_allclose(gc, h2 * mc, rtol=0, atol=2e-8 * np.abs(h2 * mc).max())
    np.testing.assert_allclose(gp, h2 * mp, rtol=0, atol=2e-8 * np.abs(h2 * mp).max())


def test_mobility_special_values():
    """M_c at pure phases and at the interface, from the definition."""
    p = PFParams(nx=4, ny=4, bc_mode="periodic")
    e = np.exp(-1 / p.sigma_surf**2)
    cases = [  # (c, phi, expected)
        (1.0, 1.0, p.MA_bulk + e * p.MA_surf),
        (0.0, 1.0, p.MB_bulk + e * p.MB_surf),
        (1.0, -1.0, e * p.MA_surf),
        (0.0, 0.0, 0.5 * p.MB_bulk + p.MB_surf),
        (1.7, 2.5, p.MA_bulk + e * p.MA_surf),     # clamped arguments
        (-0.4, -3.0, e * p.MB_surf),
        (0.5, 0.0, 0.5 * (p.MA_bulk + p.MB_bulk) / 2 + (p.MA_surf + p.MB_surf) / 2),
    ]
    for c, phi, want in cases:
        _, _, M = oracle.potentials(p, np.full((4, 4), c), np.full((4, 4), phi))
        np.testing.assert_allclose(M, want, rtol=1e-15)


# -------------------------------------------------- linearised dynamics

def _linear_matrix(p, c0, phi0, dt, lam):
    """Euler amplification matrix of (dc, dphi) for a Fourier mode of
    symbol lam, linearised about a uniform state (c0, phi0), flux off."""
    pf = (2 - phi0) * (1 + phi0) ** 2 / 4
    dpf = 3 * (1 - phi0**2) / 4
    ddpf = -1.5 * phi0
    g = c0**2 * (1 - c0) ** 2
    dg = 2 * c0 * (1 - c0) * (1 - 2 * c0)
    ddg = 2 * (1 - 6 * c0 + 6 * c0**2)
    f_cc = p.W_c * pf * ddg
    f_cp = p.W_c * dpf * dg
    f_pp = p.W_c * ddpf * g - p.W_phi * (1 - 3 * phi0**2)
    Hm = np.array([[f_cc + p.kappa_c * lam, f_cp], [f_cp, f_pp + p.kappa_phi * lam]])
    Mc = brute.mobility(p, np.array(c0), np.array(phi0))
    Mob = np.diag([float(Mc), p.M_phi])
    return np.eye(2) - dt * lam * Mob @ Hm


@pytest.mark.parametrize("c0,phi0", [(0.5, 1.0), (0.1, 1.0), (0.5, 0.3), (0.35, -0.6), (0.8, -1.0)])
def test_linear_growth_matches_closed_form(c0, phi0):
    nx, ny = 32, 32
    p = PFParams(nx=nx, ny=ny, bc_mode="periodic", flux_on=False)
    dt = 0.2 * oracle.dt_limit(p)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny))
    kx, ky = 2 * np.pi * 3 / nx, 2 * np.pi * 2 / ny
    mode = np.cos(kx * i + ky * j)
    eps_c, eps_p = 1e-7, 0.6e-7
    n = 300
    s = oracle.State(p, (c0 + eps_c * mode)[None], (phi0 + eps_p * mode)[None], np.zeros((1, ny, nx)), dt=dt)
    s.step(n)
    amp = lambda u, u0: 2 * np.sum((u - u0) * mode) / (nx * ny)
    got = np.array([amp(s.c[0], c0), amp(s.phi[0], phi0)])
    G = np.linalg.matrix_power(_linear_matrix(p, c0, phi0, dt, lam_h(kx, ky)), n)
    want = G @ np.array([eps_c, eps_p])
    scale = np.abs(want).max()
    np.testing.assert_allclose(got, want, rtol=0, atol=2e-5 * scale)


def test_biharmonic_exact_fourier_periodic():
    """W_c = 0 and species-independent mobility at phi = 1: the c update is
    linear, each Fourier mode scales by 1 - dt M kappa lam^2 per step."""
    nx, ny = 24, 16
    p = PFParams(nx=nx, ny=ny, bc_mode="periodic", flux_on=False, W_c=0.0, MB_bulk=1.0, MB_surf=5.0)
    dt = 0.2 * oracle.dt_limit(p)
    c = 0.5 + uniform01(11, np.arange(nx * ny)).reshape(1, ny, nx) - 0.5
    s = oracle.State(p, c.copy(), np.ones((1, ny, nx)), np.zeros((1, ny, nx)), dt=dt)
    n = 50
    s.step(n)
    M = p.MA_bulk + np.exp(-1 / p.sigma_surf**2) * p.MA_surf
    KX = 2 * np.pi * np.fft.fftfreq(nx)
    KY = 2 * np.pi * np.fft.fftfreq(ny)
    lam = lam_h(KX[None, :], KY[:, None])
    want = np.real(np.fft.ifft2(np.fft.fft2(c[0]) * (1 - dt * M * p.kappa_c * lam**2) ** n))
    np.testing.assert_allclose(s.c[0], want, rtol=0, atol=1e-13)
    assert np.all(s.phi == 1.0)


def test_biharmonic_exact_cosine_pvd():
    """Same linear case with PVD mirror boundaries in y: the eigenbasis is
    Fourier in x times cos(pi k (j+1/2)/ny) in y (DCT-II)."""
    from scipy.fft import dct, idct

    nx, ny = 16, 12
    p = PFParams(nx=nx, ny=ny, flux_on=False, W_c=0.0, MB_bulk=1.0, MB_surf=5.0)
    dt = 0.2 * oracle.dt_limit(p)
    c = uniform01(12, np.arange(nx * ny)).reshape(1, ny, nx)
    s = oracle.State(p, c.copy(), np.ones((1, ny, nx)), np.zeros((1, ny, nx)), dt=dt)
    n = 40
    s.step(n)
    M = p.MA_bulk + np.exp(-1 / p.sigma_surf**2) * p.MA_surf
    lam = 4 * np.sin(np.pi * np.fft.fftfreq(nx))[None, :] ** 2 + 4 * np.sin(np.pi * np.arange(ny) / (2 * ny))[:, None] ** 2
    hat = np.fft.fft(dct(c[0], type=2, axis=0, norm="ortho"), axis=1)
    hat *= (1 - dt * M * p.kappa_c * lam**2) ** n
    want = idct(np.real(np.fft.ifft(hat, axis=1)), type=2, axis=0, norm="ortho")
    np.testing.assert_allclose(s.c[0], want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("theta", [90.0, 60.0, 35.0])
def test_vapour_transport_exact_fourier(theta):
    """phi uniform makes S = 0; periodic rho is then linear: each mode scales
    by 1 - dt (D lam + i (vx sin kx h + vy sin ky h)/h)."""
    nx, ny = 20, 14
    p = PFParams(nx=nx, ny=ny, bc_mode="periodic", v0=0.9, theta_deg=theta, D_rho=0.3, h=1.3)
    dt = 0.2 * oracle.dt_limit(p)
    rho = uniform01(13, np.arange(nx * ny)).reshape(1, ny, nx)
    # uniform c and phi keep mu_phi uniform, so phi (and S = 0) stay put
    s = oracle.State(p, np.full((1, ny, nx), 0.45), np.full((1, ny, nx), 0.2), rho.copy(), dt=dt)
    n = 60
    s.step(n)
    th = np.deg2rad(theta)
    vx, vy = p.v0 * np.cos(th), -p.v0 * np.sin(th)
    KX = 2 * np.pi * np.fft.fftfreq(nx) / p.h
    KY = 2 * np.pi * np.fft.fftfreq(ny) / p.h
    lam = lam_h(KX[None, :], KY[:, None], p.h)
    sym = 1 - dt * (p.D_rho * lam + 1j * (vx * np.sin(KX[None, :] * p.h) + vy * np.sin(KY[:, None] * p.h)) / p.h)
    want = np.real(np.fft.ifft2(np.fft.fft2(rho[0]) * sym**n))
    np.testing.assert_allclose(s.rho[0], want, rtol=0, atol=1e-13)
    assert np.all(s.phi == 0.2)


# ------------------------------------------------------------- invariants

def test_conservation_flux_off_pvd():
    p = PFParams(nx=64, ny=64, flux_on=False)
    s = oracle.State.seeded(p)
    s.c[:] += 0.05 * (np.sin(np.arange(64) / 3.0)[None, :, None])  # make c non-trivial in y
    m0 = s.mass()[0]
    s.step(1000)
    m1 = s.mass()[0]
    assert abs(m1[0] - m0[0]) <= 1e-13 * abs(m0[0])
    assert abs(m1[1] - m0[1]) <= 1e-13 * abs(m0[1])
    # rho only diffuses; its change is exactly the diffusive inflow Q
    assert abs((m1[2] - m1[3]) - (m0[2] - m0[3])) <= 1e-13 * abs(m0[2])


@pytest.mark.parametrize("theta", [90.0, 55.0])
def test_phi_rho_budget_flux_on(theta):
    """h^2 sum(phi + rho) - Q and h^2 sum c are invariants of the scheme."""
    p = PFParams(nx=128, ny=128, theta_deg=theta)
    s = oracle.State.seeded(p)
    m0 = s.mass()[0]
    s.step(1000)
    m1 = s.mass()[0]
    inv0, inv1 = m0[1] + m0[2] - m0[3], m1[1] + m1[2] - m1[3]
    assert abs(inv1 - inv0) <= 1e-13 * (abs(m0[1]) + abs(m0[2]))
    assert abs(m1[0] - m0[0]) <= 1e-13 * abs(m0[0])
    assert m1[3] > 0  # vapour flows in through the top


def test_energy_decays_flux_off():
    p = PFParams(nx=128, ny=128, flux_on=False)
    s = oracle.State.seeded(p)
    E = [s.energy()[0]]
    for _ in range(1000):
        s.step(1)
        E.append(s.energy()[0])
    E = np.array(E)
    assert np.all(E[1:] <= E[:-1] + 1e-14 * np.abs(E[:-1]))
    assert E[-1] < E[0]


@pytest.mark.slow
def test_energy_decays_flux_off_long():
    p = PFParams(nx=64, ny=64, flux_on=False, c_noise=0.05)
    s = oracle.State.seeded(p)
    E0 = s.energy()[0]
    prev = E0
    for _ in range(40):
        s.step(500)
        e = s.energy()[0]
        assert e <= prev + 1e-14 * abs(prev)
        prev = e
    assert prev < E0


# ------------------------------------------------- deposition kinematics

def test_deposition_sign_and_front_speed():
    """A flat film grows: S > 0 at the interface, phi rises and rho falls
    there, and the front moves up at a speed below the inflow bound
    v0 rho_in / (2 - rho_in) of the phi+rho budget."""
    nx, ny = 4, 96
    p = PFParams(nx=nx, ny=ny, c_noise=0.0)
    s = oracle.State.seeded(p)
    phi0, rho0 = s.phi.copy(), s.rho.copy()
    s.step(1)
    j_if = int(ny / 8)
    assert s.phi[0, j_if, 0] > phi0[0, j_if, 0]
    assert s.rho[0, j_if, 0] < rho0[0, j_if, 0]

    def front(phi):
        col = phi[0, :, 0]
        k = np.nonzero((col[:-1] > 0) & (col[1:] <= 0))[0][0]
        return (k + 0.5) + col[k] / (col[k] - col[k + 1])

    s.step(5000)
    f1, t1 = front(s.phi), 5001 * s.dt
    s.step(12000)
    f2, t2 = front(s.phi), 17001 * s.dt
    V = (f2 - f1) / (t2 - t1)
    bound = p.v0 * p.rho_in / (2 - p.rho_in)
    assert 0.3 * bound < V <= 1.05 * bound


# ---------------------------------------------- independent dense assembly

@pytest.mark.parametrize("bc,theta", [("pvd", 60.0), ("pvd", 90.0), ("periodic", 40.0)])
def test_oracle_matches_dense_assembly(bc, theta):
    nx, ny = 8, 8
    p = PFParams(nx=nx, ny=ny, bc_mode=bc, theta_deg=theta, h=0.9, v0=0.7, rho_in=0.8,
                 MA_bulk=1.2, MB_bulk=0.4, MA_surf=3.0, MB_surf=1.5, sigma_surf=0.5)
    dt = 0.2 * oracle.dt_limit(p)
    c, phi, rho = random_state(5, 1, ny, nx)
    g = brute.Grid(nx, ny, p.h, periodic_y=(bc == "periodic"))
    s = oracle.State(p, c, phi, rho, dt=dt)
    u = [c[0].ravel().copy(), phi[0].ravel().copy(), rho[0].ravel().copy(), 0.0]
    for n_steps in (1, 9):
        s.step(n_steps)
        for _ in range(n_steps):
            u = list(brute.step(p, g, dt, p.v0, *u))
        for got, want in ((s.c, u[0]), (s.phi, u[1]), (s.rho, u[2])):
            np.testing.assert_allclose(got[0].ravel(), want, rtol=0, atol=1e-13 * np.abs(want).max())
        assert abs(s.Q[0] - u[3]) <= 1e-13 * max(1.0, abs(u[3]))
    E = s.energy()[0]
    assert abs(E - brute.energy(p, g, s.c[0].ravel(), s.phi[0].ravel())) <= 1e-13 * abs(E)


def test_dt_limit_is_positive_and_binding_term():
    """The stability reading's value for P0 (a check of the reading, not a pin)."""
    p = PFParams()
    lim = oracle.dt_limit(p)
    # P0: the composition Cahn-Hilliard term binds: 2 h^4 / (8 * 6 * (2 + 8))
    assert lim == pytest.approx(2.0 / 480.0, rel=1e-15)
    assert oracle.dt_limit(p.replace(v0=50.0)) == pytest.approx(2 * p.D_rho / 2500.0, rel=1e-15)
    assert oracle.dt_limit(p.replace(v0=50.0, flux_on=False)) == pytest.approx(2.0 / 480.0, rel=1e-15)


def test_batch_realisations_are_independent():
    """A batch of realisations equals separate single runs."""
    v0 = np.array([0.3, 0.8])
    c0 = np.array([0.4, 0.6])
    p = PFParams(nx=16, ny=24, batch=2, seed=4, v0_per=v0, c0_per=c0)
    dt = 0.2 * oracle.dt_limit(p)
    s = oracle.State.seeded(p, dt=dt).step(50)
    for b in range(2):
        pb = p.replace(batch=1, seed=4 + b, v0=v0[b], c0=c0[b], v0_per=None, c0_per=None)
        sb = oracle.State.seeded(pb, dt=dt).step(50)
        assert np.array_equal(sb.c[0], s.c[b]) and np.array_equal(sb.phi[0], s.phi[b])
        assert np.array_equal(sb.rho[0], s.rho[b]) and sb.Q[0] == s.Q[b]
