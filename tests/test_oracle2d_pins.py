"""Pins of the 2D oracle (fluid homogeneous in z) against what the paper's
3D formulas, its 1D model and the mathematics fix.

The paper's model is 1D; the 2D extension is derived from the same
ingredients.  Each test states what it is checked against: direct
integration of eq:force and of the 3D Shakhov and J1 formulas, the paper's
1D kernel eq:F1 and the untruncated attraction parameter eq:F2, the 1D
oracle on y-uniform states, symmetries, conservation laws and closed-form
relaxation rates.  None of these tests touches the HIP path.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import model, step1d, step2d
from oracle.model import Params, TERM_ADV, TERM_FORCE, TERM_J0, TERM_J1, FORCE_NONE
from oracle.quadrature import gauss_hermite, hermite_table


def _dt(dx, Q=8):
    return 0.2 * dx / gauss_hermite(Q)[0][-1]


# ---------------------------------------------------------------------------
# the disc kernel
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("s", [0.05, 0.25, 0.6, 0.95, 1.0, 1.3, 2.5, 4.9])
def test_kernel_2d_against_z_integral(s):
    """eq:force with n independent of z: integrate phi'(rho) s / rho along
    the z-line at in-plane distance s, outside the hard core."""
    z0 = math.sqrt(max(1.0 - s * s, 0.0))
    direct = 2 * integrate.quad(lambda z: 6 * s * (s * s + z * z) ** -4, z0, np.inf,
                                epsabs=0, epsrel=1e-13, limit=200)[0]
    kx, ky = step2d.force_kernel_2d(s, 0.0)
    assert abs(kx / direct - 1) < 1e-12 and ky == 0
    if s >= 1:
        assert abs(kx / (15 * math.pi / 8 * s ** -6) - 1) < 1e-13


def test_kernel_2d_direction_and_scaling():
    """K is radial (K_vec parallel to s_vec), scales with phi, and is
    invariant under s -> l s, sigma -> l sigma (phi'(rho) ~ phi / sigma,
    integrated along z over lengths ~ sigma)."""
    kx, ky = step2d.force_kernel_2d(0.3, 0.4, sigma=1.0, phi=1.0)
    assert abs(kx * 0.4 - ky * 0.3) < 1e-16
    kx2, ky2 = step2d.force_kernel_2d(0.3, 0.4, sigma=1.0, phi=2.5)
    assert abs(kx2 / kx - 2.5) < 1e-15
    k1 = step2d.force_kernel_2d(0.7, 0.0, sigma=1.0)[0]
    k2 = step2d.force_kernel_2d(1.4, 0.0, sigma=2.0)[0]
    assert abs(k2 / k1 - 1) < 1e-13


@pytest.mark.parametrize("x", [0.3, 0.8, 1.0, 1.7, 3.2])
def test_kernel_2d_integrates_to_paper_1d_kernel(x):
    """Integrating the disc kernel over y gives the paper's 1D EV1 kernel
    of eq:F1, 2 pi phi x (sigma / max(sigma, |x|))^6 (a fluid uniform in y
    and z)."""
    brk = [math.sqrt(1 - x * x)] if x < 1 else []
    f = lambda y: step2d.force_kernel_2d(x, y)[0]
    val = 2 * integrate.quad(f, 0, 50, points=brk or None, epsabs=0, epsrel=1e-12, limit=400)[0]
    val += 2 * integrate.quad(f, 50, np.inf, epsabs=1e-16, limit=200)[0]
    expect = 2 * math.pi * x * min(1.0, 1.0 / x) ** 6
    assert abs(val / expect - 1) < 1e-10


def test_kernel_2d_attraction_parameter_untruncated():
    """a = 1/2 int K_vec . s_vec d^2 s over the whole plane equals the
    untruncated a of eq:F2 (4 pi/3 at sigma = phi = 1)."""
    f = lambda s: 0.5 * math.pi * s * s * step2d.force_kernel_2d(s, 0.0)[0]
    a = integrate.quad(f, 0, 1, epsabs=0, epsrel=1e-13)[0] + integrate.quad(f, 1, np.inf, epsabs=0, epsrel=1e-13)[0]
    assert abs(a / model.attraction_parameter() - 1) < 1e-12


def test_disc_tables_cell_counts_and_convergence():
    """Cell-centre tables at dx = sigma/4: 45 cells in the n-bar disc, 1257
    in the force disc (r_cut = 5 sigma); the discrete attraction parameter
    converges to the truncated continuum value as dx is halved."""
    tb = step2d.Tables2D(Params(Q=4, dx=0.25, dt=1e-3))
    assert len(tb.avg_cells) == 45
    assert 2 * len(tb.force_cells) + 1 == 1257
    assert abs(sum(w for _, _, w in tb.avg_cells) - 1) < 1e-15
    f = lambda s: 0.5 * math.pi * s * s * step2d.force_kernel_2d(s, 0.0)[0]
    a_rc = integrate.quad(f, 0, 1, epsabs=0, epsrel=1e-13)[0] + integrate.quad(f, 1, 5, epsabs=0, epsrel=1e-13)[0]
    errs = [abs(step2d.attraction_parameter_2d(step2d.Tables2D(Params(Q=4, dx=dx, dt=1e-3))) - a_rc)
            for dx in (0.25, 0.125, 0.0625)]
    assert errs[0] > errs[1] > errs[2] and errs[2] / a_rc < 3e-3


def test_averaged_density_2d_converges_to_ball_average():
    """n-bar of a cosine along x tends to the ball average of Sec. II A,
    3 (sin k sigma - k sigma cos k sigma) / (k sigma)^3 cos kx, and is
    exact for uniform n."""
    N = 64
    for dx, tol in ((1 / 8, 2e-2), (1 / 16, 6e-3)):
        tb = step2d.Tables2D(Params(Q=4, dx=dx, dt=1e-3, r_cut=1.0))
        L = N * dx
        k = 2 * math.pi * 2 / L
        x = np.arange(N) * dx
        n = np.tile(np.cos(k * x), (N, 1))
        ks = k * 1.0
        transfer = 3 * (math.sin(ks) - ks * math.cos(ks)) / ks ** 3
        nb = step2d.averaged_density(n, tb)
        assert np.max(np.abs(nb - transfer * n)) < tol * abs(transfer)
    nb = step2d.averaged_density(np.full((8, 8), 0.3), tb)
    assert np.max(np.abs(nb - 0.3)) < 1e-15


# ---------------------------------------------------------------------------
# Shakhov and J1: reduction over p_z checked against the 3D formulas
# ---------------------------------------------------------------------------

class _Nodes:
    def __init__(self, v):
        self.v = v
        self.p = Params(Q=16, dx=1 / 8, dt=1e-3)


def _gauss(x, T):
    return np.exp(-x ** 2 / (2 * T)) / np.sqrt(2 * np.pi * T)


def _z_rule(T):
    z, wz = gauss_hermite(10)
    return np.sqrt(T) * z, wz


def test_shakhov_2d_reduction_matches_3d_formula():
    """The 3D Shakhov f^S of the paper, integrated over p_z (weights 1 and
    p_z^2/2) by a Gauss-Hermite rule exact for these integrands, equals the
    reduced F^S, G^S of the 2D oracle."""
    n, ux, uy, T, qx, qy, Pr = 0.4, 0.13, -0.07, 0.7, 0.021, -0.013, 0.8
    p = np.linspace(-4, 4, 9)
    pz, wz = _z_rule(T)
    FS3 = np.zeros((9, 9))
    GS3 = np.zeros((9, 9))
    for k in range(9):
        for l in range(9):
            xx, xy = p[k] - ux, p[l] - uy
            xi2 = xx ** 2 + xy ** 2 + pz ** 2
            corr = 1 + (1 - Pr) / (n * T * T) * (xi2 / (5 * T) - 1) * (xx * qx + xy * qy)
            g = n * _gauss(xx, T) * _gauss(xy, T)
            FS3[k, l] = g * np.sum(wz * corr)
            GS3[k, l] = g * np.sum(wz * 0.5 * pz ** 2 * corr)
    E = (n * _gauss(p - ux, T)[:, None] * _gauss(p - uy, T)[None, :])[:, :, None, None]
    a = lambda v: np.array([[v]])
    m = dict(n=a(n), ux=a(ux), uy=a(uy), T=a(T), qx=a(qx), qy=a(qy), Pr=a(Pr))
    FS, GS = step2d.shakhov(E, m, _Nodes(p))
    assert np.allclose(FS[:, :, 0, 0], FS3, rtol=1e-13, atol=1e-16)
    assert np.allclose(GS[:, :, 0, 0], GS3, rtol=1e-13, atol=1e-16)


def test_j1_2d_reduction_matches_3d_formula():
    """eq:J1 with in-plane gradients (full grad-u tensor), integrated over
    p_z, against the reduced J1F, J1G of the 2D oracle."""
    n, ux, uy, T, chi = 0.35, -0.08, 0.05, 0.62, 1.9
    Ax, Ay, Bx, By = 0.3, -0.11, -0.2, 0.07
    Uxx, Uxy, Uyx, Uyy = 0.05, -0.03, 0.02, 0.04   # U_ij = d_i u_j
    b = model.excluded_volume(1.0)
    p = np.linspace(-4, 4, 9)
    pz, wz = _z_rule(T)
    J1F3 = np.zeros((9, 9))
    J1G3 = np.zeros((9, 9))
    for k in range(9):
        for l in range(9):
            xx, xy = p[k] - ux, p[l] - uy
            zeta2 = (xx ** 2 + xy ** 2 + pz ** 2) / (2 * T)
            zz = (xx * xx * Uxx + xx * xy * Uxy + xy * xx * Uyx + xy * xy * Uyy) / (2 * T)
            brace = (xx * (Ax + 0.6 * (zeta2 - 2.5) * Bx) + xy * (Ay + 0.6 * (zeta2 - 2.5) * By)
                     + 0.4 * (2 * zz + (zeta2 - 2.5) * (Uxx + Uyy)))
            g = -b * n * chi * n * _gauss(xx, T) * _gauss(xy, T)
            J1F3[k, l] = g * np.sum(wz * brace)
            J1G3[k, l] = g * np.sum(wz * 0.5 * pz ** 2 * brace)
    E = (n * _gauss(p - ux, T)[:, None] * _gauss(p - uy, T)[None, :])[:, :, None, None]
    a = lambda v: np.array([[v]])
    m = dict(n=a(n), ux=a(ux), uy=a(uy), T=a(T), chi=a(chi), Ax=a(Ax), Ay=a(Ay), Bx=a(Bx), By=a(By),
             Uxx=a(Uxx), Uxy=a(Uxy), Uyx=a(Uyx), Uyy=a(Uyy))
    J1F, J1G = step2d.j1_terms(E, m, _Nodes(p))
    assert np.allclose(J1F[:, :, 0, 0], J1F3, rtol=1e-12, atol=1e-15)
    assert np.allclose(J1G[:, :, 0, 0], J1G3, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------
# reduction to the 1D model
# ---------------------------------------------------------------------------

def _y_uniform_state(N, Q, tb2, seed, n_uniform=True):
    """y-uniform 2D state with zero y-momentum at every node (perturbation
    symmetric under p_y -> -p_y) and, optionally, uniform density."""
    rng = np.random.default_rng(seed)
    x = np.arange(N) / N
    n = 0.3 * (1 + (0 * x if n_uniform else 0.05 * np.sin(2 * np.pi * x)))
    ux = 0.06 * np.cos(2 * np.pi * x)
    T = 0.6 * (1 + 0.05 * np.sin(2 * np.pi * 2 * x))
    F, G = step2d.initial_state(n[None, :].repeat(4, 0), ux[None, :].repeat(4, 0), 0.0,
                                T[None, :].repeat(4, 0), tb2)
    pert = rng.standard_normal((Q, Q, 1, N))
    pert = pert + pert[:, ::-1]
    F = F * (1 + 0.02 * pert)
    G = G * (1 + 0.01 * pert[::-1])
    if n_uniform:
        F = F * (n[None, None] / F.sum((0, 1)))[:, :]
    return F, G


def _reduce(F, G, v):
    vy = v[None, :, None]
    return F[:, :, 0, :].sum(1), (0.5 * vy ** 2 * F[:, :, 0, :] + G[:, :, 0, :]).sum(1)


def test_y_uniform_rhs_reduces_to_1d_rhs():
    """For a y-uniform state with uniform density and no y-momentum, the 2D
    force, Shakhov and J1 terms summed over p_y (weights 1 and p_y^2/2)
    equal the 1D oracle's terms on the reduced state (the disc n-bar and
    disc force then agree with the 1D ones: n-bar = n, F = g_ext)."""
    N, Q = 32, 8
    mask = TERM_FORCE | TERM_J0 | TERM_J1
    kw = dict(Q=Q, dx=0.25, dt=_dt(0.25), term_mask=mask, g_ext=0.05)
    tb2 = step2d.Tables2D(Params(**kw))
    tb1 = step1d.Tables(Params(**kw))
    F, G = _y_uniform_state(N, Q, tb2, seed=3)
    F1, G1 = _reduce(F, G, tb2.v)
    L2F, L2G = step2d.rhs(F, G, tb2)
    assert np.max(np.abs(L2F - L2F[:, :, :1])) == 0
    R2F, R2G = _reduce(L2F, L2G, tb2.v)
    L1F, L1G = step1d.rhs(F1, G1, tb1)
    assert np.max(np.abs(R2F - L1F)) < 1e-13 * np.max(np.abs(L1F))
    assert np.max(np.abs(R2G - L1G)) < 1e-13 * np.max(np.abs(L1G))


def test_y_uniform_advection_is_1d_weno():
    """Advection of a y-uniform state: the y-sweep vanishes exactly and the
    x-sweep is the 1D oracle's WENO advection of each p_y row."""
    N, Q = 40, 8
    kw = dict(Q=Q, dx=0.25, dt=_dt(0.25), term_mask=TERM_ADV)
    tb2 = step2d.Tables2D(Params(**kw))
    tb1 = step1d.Tables(Params(**kw))
    rng = np.random.default_rng(5)
    A = 1 + 0.3 * rng.random((Q, Q, 1, N))
    F = np.repeat(A, 3, axis=2)
    adv = step2d.advection(F, tb2)
    for l in range(Q):
        ref = step1d.weno5_advection(A[:, l, 0, :], tb1)
        for y in range(3):
            assert np.max(np.abs(adv[:, l, y, :] - ref)) <= 1e-15 * np.max(np.abs(ref))


# ---------------------------------------------------------------------------
# symmetries
# ---------------------------------------------------------------------------

def _random_2d(N=16, Q=8, dx=0.25, seed=7, **kw):
    tb = step2d.Tables2D(Params(Q=Q, dx=dx, dt=_dt(dx, Q), **kw))
    rng = np.random.default_rng(seed)
    n = 0.3 * (1 + 0.05 * rng.standard_normal((N, N)))
    ux = 0.04 * rng.standard_normal((N, N))
    uy = 0.04 * rng.standard_normal((N, N))
    T = 0.6 * (1 + 0.03 * rng.standard_normal((N, N)))
    F, G = step2d.initial_state(n, ux, uy, T, tb)
    wn = tb.w / tb.w.max()
    F = F * (1 + 0.02 * rng.standard_normal(F.shape) * wn[:, None, None, None] * wn[None, :, None, None])
    G = G * (1 + 0.02 * rng.standard_normal(G.shape) * wn[:, None, None, None] * wn[None, :, None, None])
    return F, G, tb


def test_rhs_symmetric_under_axis_swap():
    """Swapping x <-> y together with p_x <-> p_y commutes with the RHS."""
    F, G, tb = _random_2d()
    LF, LG = step2d.rhs(F, G, tb)
    sw = lambda a: a.transpose(1, 0, 3, 2)
    SF, SG = step2d.rhs(sw(F), sw(G), tb)
    assert np.max(np.abs(SF - sw(LF))) < 1e-13 * np.max(np.abs(LF))
    assert np.max(np.abs(SG - sw(LG))) < 1e-13 * np.max(np.abs(LG))


def test_rhs_symmetric_under_reflection():
    """Reflecting x -> -x (node i -> -i mod N) together with p_x -> -p_x
    commutes with the RHS (upwind mirror of WENO, odd force kernel)."""
    F, G, tb = _random_2d(seed=8)
    N = F.shape[-1]
    idx = (-np.arange(N)) % N
    rf = lambda a: a[::-1][:, :, :, idx]
    LF, LG = step2d.rhs(F, G, tb)
    RF, RG = step2d.rhs(rf(F), rf(G), tb)
    assert np.max(np.abs(RF - rf(LF))) < 1e-13 * np.max(np.abs(LF))
    assert np.max(np.abs(RG - rf(LG))) < 1e-13 * np.max(np.abs(LG))


# ---------------------------------------------------------------------------
# whole step
# ---------------------------------------------------------------------------

def test_equilibrium_2d_moments():
    """The tensor Hermite equilibrium with G = T/2 E reproduces n, u, T and
    has no heat flux."""
    tb = step2d.Tables2D(Params(Q=16, dx=0.25, dt=1e-3))
    n = np.linspace(0.1, 0.6, 6).reshape(2, 3)
    ux = np.linspace(-0.2, 0.2, 6).reshape(2, 3)
    uy = np.linspace(0.15, -0.1, 6).reshape(2, 3)
    T = np.linspace(0.5, 0.9, 6).reshape(2, 3)
    F, G = step2d.initial_state(n, ux, uy, T, tb)
    n2, ux2, uy2, T2, qx, qy = step2d.moments(F, G, tb)
    assert np.allclose(n2, n, rtol=1e-14) and np.allclose(ux2, ux, atol=1e-14) and np.allclose(uy2, uy, atol=1e-14)
    assert np.allclose(T2, T, rtol=1e-13) and np.max(np.abs(qx)) < 1e-14 and np.max(np.abs(qy)) < 1e-14


def test_uniform_maxwellian_2d_is_stationary():
    tb = step2d.Tables2D(Params(Q=8, dx=0.25, dt=_dt(0.25)))
    F, G = step2d.initial_state(np.full((12, 12), 0.3), 0.0, 0.0, np.full((12, 12), 0.6), tb)
    F1, G1 = step2d.run(F, G, tb, 5)
    assert np.max(np.abs(F1 - F)) <= 1e-14 * np.max(F)
    assert np.max(np.abs(G1 - G)) <= 1e-14 * np.max(G)


def test_conservation_2d():
    """Periodic 2D system: mass and both momentum components conserved to
    round-off; the energy changes by the work of the mean-field force,
    dt (W0/6 + W1/6 + 2 W2/3), W = sum n (u_x F_x + u_y F_y)."""
    F, G, tb = _random_2d(N=20)
    vx = tb.v[:, None, None, None]
    vy = tb.v[None, :, None, None]
    for _ in range(2):
        mass0 = F.sum()
        scale = np.sum((np.abs(vx) + np.abs(vy)) * F)
        px0, py0 = (vx * F).sum(), (vy * F).sum()
        en0 = (0.5 * (vx ** 2 + vy ** 2) * F + G).sum()
        work = []
        Fs, Gs = F, G
        for a, b in step2d.RK3_COEFFS:
            m = step2d.node_fields(Fs, Gs, tb)
            work.append(np.sum(m["n"] * (m["ux"] * m["Fx"] + m["uy"] * m["Fy"])))
            LF, LG = step2d.rhs(Fs, Gs, tb)
            Fs, Gs = a * F + b * (Fs + tb.p.dt * LF), a * G + b * (Gs + tb.p.dt * LG)
        F1, G1 = step2d.rk3_step(F, G, tb)
        assert np.array_equal(F1, Fs)
        assert abs(F1.sum() - mass0) < 1e-13 * mass0
        assert abs((vx * F1).sum() - px0) < 1e-13 * scale
        assert abs((vy * F1).sum() - py0) < 1e-13 * scale
        en1 = (0.5 * (vx ** 2 + vy ** 2) * F1 + G1).sum()
        budget = tb.p.dt * (work[0] / 6 + work[1] / 6 + 2 * work[2] / 3)
        assert abs(en1 - en0 - budget) < 1e-13 * en0
        F, G = F1, G1


def test_homogeneous_relaxation_2d_closed_form():
    """Uniform non-equilibrium state: the shear stress P_xy decays by
    R(-nu dt) and the heat flux q_x by R(-Pr nu dt) per step,
    R(z) = 1 + z + z^2/2 + z^3/6."""
    Q, N = 8, 4
    tb = step2d.Tables2D(Params(Q=Q, dx=0.25, dt=0.05))
    n0, T0 = 0.45, 0.7
    F, G = step2d.initial_state(np.full((N, N), n0), 0.0, 0.0, np.full((N, N), T0), tb)
    He = hermite_table(tb.v, 3)
    eps = 1e-3
    wk = tb.w[:, None, None, None]
    wl = tb.w[None, :, None, None]
    F = F + eps * (wk * He[1][:, None, None, None]) * (wl * He[1][None, :, None, None])
    F = F + 0.5 * eps * (wk * He[3][:, None, None, None]) * wl
    m = step2d.node_fields(F, G, tb)
    nu, Pr = m["nu"][0, 0], m["Pr"][0, 0]
    R = lambda z: 1 + z + z * z / 2 + z ** 3 / 6
    vx = tb.v[:, None, None, None]
    vy = tb.v[None, :, None, None]
    pxy0 = (vx * vy * F).sum((0, 1))[0, 0]
    qx0 = m["qx"][0, 0]
    F1, G1 = step2d.rk3_step(F, G, tb)
    n1, ux1, uy1, T1, qx1, qy1 = step2d.moments(F1, G1, tb)
    pxy1 = (vx * vy * F1).sum((0, 1))[0, 0]
    assert abs(pxy1 / pxy0 - R(-nu * tb.p.dt)) < 1e-11
    assert abs(qx1[0, 0] / qx0 - R(-Pr * nu * tb.p.dt)) < 1e-11


def test_uniform_external_force_2d():
    """Force term alone with a uniform acceleration g along x: u_x grows as
    g t, u_y and T stay fixed."""
    tb = step2d.Tables2D(Params(Q=8, dx=0.25, dt=0.01, term_mask=TERM_FORCE, force_model=FORCE_NONE, g_ext=0.2))
    F, G = step2d.initial_state(np.full((4, 4), 0.3), 0.0, 0.0, np.full((4, 4), 0.6), tb)
    F1, G1 = step2d.run(F, G, tb, 20)
    n, ux, uy, T, qx, qy = step2d.moments(F1, G1, tb)
    assert np.allclose(ux, 0.2 * 20 * 0.01, rtol=1e-12)
    assert np.max(np.abs(uy)) < 1e-14 and np.allclose(T, 0.6, rtol=1e-12)


def test_isothermal_2d_rhs_equals_thermal_at_uniform_temperature():
    """2D isothermal mode: with the moment temperature uniform and equal to
    T_iso the right-hand side is the thermal one."""
    tb = step2d.Tables2D(Params(Q=8, dx=0.25, dt=_dt(0.25)))
    tbi = step2d.Tables2D(Params(Q=8, dx=0.25, dt=_dt(0.25), T_iso=0.6))
    rng = np.random.default_rng(4)
    N = 12
    n = 0.3 * (1 + 0.05 * rng.standard_normal((N, N)))
    ux = 0.03 * rng.standard_normal((N, N))
    uy = 0.03 * rng.standard_normal((N, N))
    F, G = step2d.initial_state(n, ux, uy, np.full((N, N), 0.6), tb)
    LF, LG = step2d.rhs(F, G, tb)
    LFi, LGi = step2d.rhs(F, G, tbi)
    assert np.max(np.abs(LFi - LF)) < 1e-12 * np.max(np.abs(LF))
    assert np.max(np.abs(LGi - LG)) < 1e-12 * np.max(np.abs(LG))


@pytest.mark.parametrize("mx,my", [(1, 3), (7, 2), (15, 11)])
def test_gradients_2d_exact_discrete_symbol(mx, my):
    """Dx and Dy are the 4th-order central stencil along x (last axis) and
    y: on cos(kx x + ky y) each gives -(8 sin t - sin 2t) / (6 dx) sin(...)
    with t = k dx of its own axis, exactly."""
    ny, nx, dx = 24, 32, 0.25
    y, x = np.meshgrid(np.arange(ny) * dx, np.arange(nx) * dx, indexing="ij")
    tx, ty = 2 * np.pi * mx / nx, 2 * np.pi * my / ny
    g = np.cos(tx / dx * x + ty / dx * y)
    sn = np.sin(tx / dx * x + ty / dx * y)
    sym = lambda t: (8 * np.sin(t) - np.sin(2 * t)) / (6 * dx)
    assert np.max(np.abs(step2d.Dx(g, dx) + sym(tx) * sn)) < 1e-13
    assert np.max(np.abs(step2d.Dy(g, dx) + sym(ty) * sn)) < 1e-13


def test_momentum_derivative_2d_acts_on_its_own_axis():
    """On a separable velocity profile f[k, l] = g[k] h[l] (per node), the
    x-derivative is (Dp g)[k] h[l] and the y-derivative g[k] (Dp h)[l]; Dp is
    not symmetric, so a transposed or swapped operand fails."""
    tb = step2d.Tables2D(Params(Q=8, dx=0.25, dt=1e-3))
    Q = 8
    rng = np.random.default_rng(11)
    g, h = rng.standard_normal((Q, 3)), rng.standard_normal((Q, 3))
    f = g[:, None, :] * h[None, :, :]
    Dp = tb.Dp
    assert np.max(np.abs(Dp - Dp.T)) > 1e-3
    ref_x = np.stack([sum(Dp[k, j] * g[j] for j in range(Q)) for k in range(Q)])[:, None, :] * h[None, :, :]
    ref_y = g[:, None, :] * np.stack([sum(Dp[l, j] * h[j] for j in range(Q)) for l in range(Q)])[None, :, :]
    assert np.max(np.abs(step2d.dp_x(f, tb) - ref_x)) < 1e-12
    assert np.max(np.abs(step2d.dp_y(f, tb) - ref_y)) < 1e-12
