"""One time step of the 2D extension of the EV-FDLB model (test
infrastructure).

The paper solves the 1D model (fluid homogeneous in y and z, Sec. III) and
names the extension to two or three dimensions as a goal in its conclusions.
This module is the same method for a fluid homogeneous in z only, built from
the same ingredients.  The reading is stated here and derived from the paper's 3D
formulas; the tests pin the reductions against direct integration of those
formulas.

State: F(x, y, p_x, p_y) = integral f dp_z and G = integral p_z^2/2 f dp_z on
the tensor-product Gauss-Hermite set (p_x, p_y) = (p_k, p_l), stored as arrays
of shape (Q, Q, Ny, Nx) (index k of p_x, index l of p_y, then y, x), periodic
in x and y with spacing dx.

Right-hand side (eq:enskog_approx with the mean field, reduced over p_z):
    dF/dt = -p_x dF/dx - p_y dF/dy - F_x dF/dp_x - F_y dF/dp_y
            - nu (F - F^S) + J1F                       (G likewise)
with
    moments   n, n u = sum p F, 3/2 n T = sum (|xi|^2/2 F + G),
              q = sum xi (|xi|^2/2 F + G),   xi = (p_x - u_x, p_y - u_y);
    Shakhov   F^S = E [1 + s (xi.q)(theta - 4)],
              G^S = T/2 E [1 + s (xi.q)(theta - 2)],
              theta = |xi|^2/T, s = (1 - Pr)/(5 n T^2);
    J1        J1F = -b n chi E {xi.[A + 0.3 (theta-4) B] + 0.4 [xi_i xi_j d_i u_j / T
                                 + 1/2 (theta-4) div u]},
              J1G = -b n chi T/2 E {xi.[A + 0.3 (theta-2) B] + 0.4 [xi_i xi_j d_i u_j / T
                                 + 1/2 (theta-2) div u]},
              A = grad ln(n^2 chi T), B = grad ln T;
    E         tensor product of the 1D Hermite equilibria: n e_k(u_x) e_l(u_y);
    force     the z-integrated mean-field kernel (Vlasov force eq:force with n
              independent of z), summed over grid cells within r_cut;
    nbar      the ball average of Sec. II A, z-integrated: weights
              2 sqrt(sigma^2 - s^2) over cells with s < sigma.
Discretisation: WENO-5 along each axis, 4th-order central gradients along
each axis, TVD-RK3.

Readings (the paper is 1D): cell-centre rule for the disc sums (composite
Simpson does not apply on a disc), n-bar weights renormalised to sum 1, force
pairs +-s summed antisymmetrically.  The tests pin these discretisations by
their convergence to the continuum integrals, the reduced collision terms by
integration of the 3D formulas, and the whole right-hand side by its
reduction to the 1D step on y-uniform states.
"""
import numpy as np

from . import model
from .model import Params, TERM_ADV, TERM_FORCE, TERM_J0, TERM_J1, FORCE_EV1, FORCE_NONE
from .quadrature import gauss_hermite, equilibrium_matrix, momentum_derivative_matrix, hermite_moments_maxwellian
from .step1d import weno5_reconstruct


def force_kernel_2d(sx, sy, sigma=1.0, phi=1.0):
    """z-integrated force kernel of the Sutherland tail (gamma = 6) for an
    in-plane separation s_vec = (sx, sy): the force eq:force exerts on a
    particle from a line of density along z at in-plane distance s, with the
    part of the line inside the hard core (rho < sigma) excluded.  With
    z = s tan(t) the z-integral of 6 phi sigma^6 s rho^-8 becomes
        K(s) = 12 phi sigma^6 s^-6 int_0^psi sin^6 t dt,
    psi = arcsin(s / sigma) for s < sigma and pi/2 otherwise, so that
    K = (15 pi / 8) phi sigma^6 s^-6 outside the core.  The t-integral is
    taken by 24-point Gauss-Legendre (exact to rounding for this entire
    integrand), which avoids the cancellation of the closed-form primitive
    at small s."""
    sx = np.asarray(sx, dtype=np.float64)
    sy = np.asarray(sy, dtype=np.float64)
    s = np.hypot(sx, sy)
    psi = np.where(s < sigma, np.arcsin(np.minimum(s / sigma, 1.0)), np.pi / 2)
    t, wt = np.polynomial.legendre.leggauss(24)
    nodes = 0.5 * psi[..., None] * (t + 1)
    integral = 0.5 * psi * np.sum(wt * np.sin(nodes) ** 6, axis=-1)
    safe = np.where(s > 0, s, 1.0)
    mag = np.where(s > 0, 12.0 * phi * sigma ** 6 * safe ** -7 * integral, 0.0)
    return mag * sx, mag * sy


class Tables2D:
    """Quadrature and stencil tables of one 2D parameter set (gamma = 6)."""

    def __init__(self, p: Params):
        if p.gamma != 6.0:
            raise ValueError("the 2D kernel is tabulated for gamma = 6")
        self.p = p
        self.v, self.w = gauss_hermite(p.Q)
        self.Meq = equilibrium_matrix(self.v, self.w)
        self.Dp = momentum_derivative_matrix(self.v, self.w)
        Ms = int(np.ceil(p.sigma_ref / p.dx))
        cells = []
        for j in range(-Ms, Ms + 1):
            for i in range(-Ms, Ms + 1):
                s = p.dx * np.hypot(i, j)
                if s < p.sigma_ref:
                    cells.append((j, i, 2.0 * np.sqrt(p.sigma ** 2 - s ** 2)))
        tot = sum(c[2] for c in cells)
        self.avg_cells = [(j, i, wgt / tot) for j, i, wgt in cells]
        MF = int(round(p.r_cut / p.dx))
        fc = []
        for j in range(-MF, MF + 1):
            for i in range(-MF, MF + 1):
                s2 = i * i + j * j
                # one representative of each +-s pair (i > 0, or i == 0 and j > 0)
                if s2 == 0 or s2 * p.dx ** 2 > p.r_cut ** 2 + 1e-12 or not (i > 0 or (i == 0 and j > 0)):
                    continue
                kx, ky = force_kernel_2d(i * p.dx, j * p.dx, p.sigma, p.phi)
                fc.append((j, i, kx * p.dx ** 2, ky * p.dx ** 2))
        self.force_cells = fc


def attraction_parameter_2d(tb: Tables2D):
    """a_disc = 1/2 sum over cells of K_x s_x dx^2 (long-wave limit
    F -> 2 a grad n of the discrete force)."""
    return sum(cx * i * tb.p.dx for j, i, cx, cy in tb.force_cells)


def sh(a, dy, dx):
    """a[..., y + dy, x + dx] on the periodic grid."""
    return np.roll(np.roll(a, -dy, axis=-2), -dx, axis=-1)


def moments(F, G, tb):
    vx = tb.v[:, None, None, None]
    vy = tb.v[None, :, None, None]
    n = F.sum((0, 1))
    ux = (vx * F).sum((0, 1)) / n
    uy = (vy * F).sum((0, 1)) / n
    xx = vx - ux
    xy = vy - uy
    e = 0.5 * (xx ** 2 + xy ** 2) * F + G
    T = (2.0 / 3.0) * e.sum((0, 1)) / n
    qx = (xx * e).sum((0, 1))
    qy = (xy * e).sum((0, 1))
    return n, ux, uy, T, qx, qy


def averaged_density(n, tb):
    out = np.zeros_like(n, dtype=np.result_type(n, tb.p.sigma))
    for j, i, w in tb.avg_cells:
        out = out + w * sh(n, j, i)
    return out


def vlasov_force(n, tb):
    Fx = np.zeros_like(n, dtype=np.result_type(n, tb.p.phi, tb.p.sigma))
    Fy = np.zeros_like(Fx)
    if tb.p.force_model == FORCE_EV1:
        for j, i, cx, cy in tb.force_cells:
            d = sh(n, j, i) - sh(n, -j, -i)
            Fx = Fx + cx * d
            Fy = Fy + cy * d
    elif tb.p.force_model != FORCE_NONE:
        raise ValueError("2D: EV1 or no force")
    return Fx + tb.p.g_ext, Fy


def Dx(g, dx):
    return (sh(g, 0, -2) - 8 * sh(g, 0, -1) + 8 * sh(g, 0, 1) - sh(g, 0, 2)) / (12 * dx)


def Dy(g, dx):
    return (sh(g, -2, 0) - 8 * sh(g, -1, 0) + 8 * sh(g, 1, 0) - sh(g, 2, 0)) / (12 * dx)


def equilibrium(n, ux, uy, T, tb):
    Q = tb.p.Q
    ex = tb.Meq @ hermite_moments_maxwellian(np.ones_like(n), ux, T, Q).reshape(Q, -1)
    ey = tb.Meq @ hermite_moments_maxwellian(np.ones_like(n), uy, T, Q).reshape(Q, -1)
    shp = n.shape
    return n[None, None] * ex.reshape((Q, 1) + shp) * ey.reshape((1, Q) + shp)


def node_fields(F, G, tb):
    p = tb.p
    n, ux, uy, T, qx, qy = moments(F, G, tb)
    if p.T_iso:
        T = np.full_like(T, p.T_iso)
    nbar = averaged_density(n, tb)
    chi = model.contact_value(nbar, p.sigma)
    Fx, Fy = vlasov_force(n, tb)
    nu = model.collision_rate(n, T, chi, p.sigma)
    Pr = model.prandtl(n, chi, p.sigma)
    X = n ** 2 * chi * T
    return dict(n=n, ux=ux, uy=uy, T=T, qx=qx, qy=qy, nbar=nbar, chi=chi, Fx=Fx, Fy=Fy, nu=nu, Pr=Pr, X=X,
                Ax=Dx(X, p.dx) / X, Ay=Dy(X, p.dx) / X, Bx=Dx(T, p.dx) / T, By=Dy(T, p.dx) / T,
                Uxx=Dx(ux, p.dx), Uxy=Dx(uy, p.dx), Uyx=Dy(ux, p.dx), Uyy=Dy(uy, p.dx))


def shakhov(E, m, tb):
    vx = tb.v[:, None, None, None]
    vy = tb.v[None, :, None, None]
    xx, xy = vx - m["ux"], vy - m["uy"]
    T = m["T"]
    th = (xx ** 2 + xy ** 2) / T
    s = (1 - m["Pr"]) / (5 * m["n"] * T ** 2)
    xq = xx * m["qx"] + xy * m["qy"]
    return E * (1 + s * xq * (th - 4)), 0.5 * T * E * (1 + s * xq * (th - 2))


def j1_terms(E, m, tb):
    vx = tb.v[:, None, None, None]
    vy = tb.v[None, :, None, None]
    xx, xy = vx - m["ux"], vy - m["uy"]
    T = m["T"]
    th = (xx ** 2 + xy ** 2) / T
    b = model.excluded_volume(tb.p.sigma)
    pre = -b * m["n"] * m["chi"]
    xxu = (xx * xx * m["Uxx"] + xx * xy * m["Uxy"] + xy * xx * m["Uyx"] + xy * xy * m["Uyy"]) / T
    div = m["Uxx"] + m["Uyy"]
    xA = xx * m["Ax"] + xy * m["Ay"]
    xB = xx * m["Bx"] + xy * m["By"]
    J1F = pre * E * (xA + 0.3 * (th - 4) * xB + 0.4 * (xxu + 0.5 * (th - 4) * div))
    J1G = pre * 0.5 * T * E * (xA + 0.3 * (th - 2) * xB + 0.4 * (xxu + 0.5 * (th - 2) * div))
    return J1F, J1G


def weno_flux_axis(f, pk, axis, tb):
    """-p (fhat_{i+1/2} - fhat_{i-1/2}) / dx along one grid axis (-1: x,
    -2: y) of a (Ny, Nx) array, upwind by the sign of p."""
    eps = tb.p.weno_eps

    def s(a, j):
        return np.roll(a, -j, axis=axis)

    if pk > 0:
        fh = weno5_reconstruct(s(f, -2), s(f, -1), f, s(f, 1), s(f, 2), eps)
    else:
        fh = weno5_reconstruct(s(f, 3), s(f, 2), s(f, 1), f, s(f, -1), eps)
    return -pk * (fh - s(fh, -1)) / tb.p.dx


def advection(f, tb):
    out = np.zeros_like(f)
    Q = tb.p.Q
    for k in range(Q):
        for l in range(Q):
            out[k, l] = weno_flux_axis(f[k, l], tb.v[k], -1, tb) + weno_flux_axis(f[k, l], tb.v[l], -2, tb)
    return out


def dp_x(f, tb):
    return np.einsum("ab,bl...->al...", tb.Dp, f)


def dp_y(f, tb):
    return np.einsum("ab,kb...->ka...", tb.Dp, f)


def rhs(F, G, tb):
    p = tb.p
    m = node_fields(F, G, tb)
    E = equilibrium(m["n"], m["ux"], m["uy"], m["T"], tb)
    LF = np.zeros_like(F)
    LG = np.zeros_like(G)
    if p.term_mask & TERM_ADV:
        LF = LF + advection(F, tb)
        LG = LG + advection(G, tb)
    if p.term_mask & TERM_FORCE:
        LF = LF - m["Fx"] * dp_x(F, tb) - m["Fy"] * dp_y(F, tb)
        LG = LG - m["Fx"] * dp_x(G, tb) - m["Fy"] * dp_y(G, tb)
    if p.term_mask & TERM_J0:
        FS, GS = shakhov(E, m, tb)
        LF = LF - m["nu"] * (F - FS)
        LG = LG - m["nu"] * (G - GS)
    if p.term_mask & TERM_J1:
        J1F, J1G = j1_terms(E, m, tb)
        LF = LF + J1F
        LG = LG + J1G
    return LF, LG


RK3_COEFFS = ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0))


def rk3_step(F, G, tb):
    dt = tb.p.dt
    Fs, Gs = F, G
    for a, b in RK3_COEFFS:
        LF, LG = rhs(Fs, Gs, tb)
        Fs, Gs = a * F + b * (Fs + dt * LF), a * G + b * (Gs + dt * LG)
    return Fs, Gs


def run(F, G, tb, nsteps):
    for _ in range(nsteps):
        F, G = rk3_step(F, G, tb)
    return F, G


def initial_state(n, ux, uy, T, tb):
    """F = E(n, u, T), G = T/2 E (the p_z energy of the Maxwellian)."""
    n = np.asarray(n)
    shp = n.shape
    ux = np.broadcast_to(np.asarray(ux, dtype=np.result_type(n, ux)), shp)
    uy = np.broadcast_to(np.asarray(uy, dtype=np.result_type(n, uy)), shp)
    T = np.broadcast_to(np.asarray(T, dtype=np.result_type(n, T)), shp)
    E = equilibrium(n, ux, uy, T, tb)
    return E, 0.5 * T * E
