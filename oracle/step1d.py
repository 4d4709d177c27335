"""One time step of the reduced 1D EV-FDLB model (test infrastructure).

The fluid is homogeneous in y and z (Sec. III), so the state at grid node
x_i is a pair of reduced distributions on the Gauss-Hermite nodes p_k:

    F_k(x) = integral f dp_y dp_z,   G_k(x) = integral (p_y^2+p_z^2)/2 f dp_y dp_z

stored as arrays of shape (Q, N) on a periodic grid of spacing dx.

The right-hand side follows the simplified evolution equation
(eq:enskog_approx with the EV1 force eq:F1, i.e. eq:ev1):

    dF/dt = -p dF/dx - Fx (dF/dp) - nu (F - F^S) + J1F
    dG/dt = -p dG/dx - Fx (dG/dp) - nu (G - G^S) + J1G

discretised with the schemes the paper lists (Sec. III): WENO-5 advection,
4th-order central differences for the gradients in J1, composite Simpson
for the force integral, TVD Runge-Kutta 3 in time.  The routines below are
that right-hand side in the paper's order: moments, averaged density and
contact value, Vlasov force, transport, gradients, Hermite equilibrium,
Shakhov distribution, J1, momentum derivative, advection, combine.

All node fields are re-evaluated at every Runge-Kutta stage.
"""
import numpy as np

from . import model
from .model import (Params, TERM_ADV, TERM_FORCE, TERM_J0, TERM_J1,
                    FORCE_EV1, FORCE_EV2, FORCE_NONE)
from .quadrature import (gauss_hermite, equilibrium_matrix,
                         momentum_derivative_matrix, hermite_moments_maxwellian)


class Tables:
    """Quadrature and stencil tables of one parameter set."""

    def __init__(self, p: Params):
        self.p = p
        self.v, self.w = gauss_hermite(p.Q)
        self.Meq = equilibrium_matrix(self.v, self.w)
        self.Dp = momentum_derivative_matrix(self.v, self.w)
        self.s_avg = model.averaging_weights(p)
        self.c_force = model.force_weights(p)


def shift(a, j):
    """a[..., i + j] on the periodic grid."""
    return np.roll(a, -j, axis=-1)


# --- macroscopic moments (Sec. II B, moments equation; Shakhov heat flux) ---

def moments(F, G, tb: Tables):
    """n, u, T, q of the reduced distributions.

    n = int f,  n u = int p f,  3/2 n T = int xi^2/2 f,
    q = int xi^2/2 xi f  (x-component), with xi = p - u and
    xi^2 = xi_x^2 + p_y^2 + p_z^2, so that
    3/2 n T = sum_k (xi_k^2/2 F_k + G_k) and q = sum_k xi_k (xi_k^2/2 F_k + G_k).
    """
    v = tb.v[:, None]
    n = F.sum(0)
    u = (v * F).sum(0) / n
    xi = v - u[None, :]
    e = 0.5 * xi ** 2 * F + G
    T = (2.0 / 3.0) * e.sum(0) / n
    q = (xi * e).sum(0)
    return n, u, T, q


# --- Fischer-Methfessel averaged density and contact value ---

def averaged_density(n, tb: Tables):
    """nbar_i = sum_j s_j n_{i+j} (see model.averaging_weights)."""
    Ms = (len(tb.s_avg) - 1) // 2
    out = np.zeros_like(n, dtype=np.result_type(n, tb.s_avg))
    for j in range(-Ms, Ms + 1):
        out = out + tb.s_avg[j + Ms] * shift(n, j)
    return out


# --- self-consistent (Vlasov) force ---

def vlasov_force_ev1(n, tb: Tables):
    """eq:F1 by composite Simpson: F_i = sum_{j>=1} c_j (n_{i+j} - n_{i-j})."""
    out = np.zeros_like(n, dtype=np.result_type(n, tb.c_force))
    for j in range(1, len(tb.c_force) + 1):
        out = out + tb.c_force[j - 1] * (shift(n, j) - shift(n, -j))
    return out


def central_gradient(g, dx):
    """4th-order central difference
    (g_{i-2} - 8 g_{i-1} + 8 g_{i+1} - g_{i+2}) / (12 dx)."""
    return (shift(g, -2) - 8.0 * shift(g, -1) + 8.0 * shift(g, 1) - shift(g, 2)) / (12.0 * dx)


def third_derivative(g, dx):
    """5-point third derivative
    (-g_{i-2} + 2 g_{i-1} - 2 g_{i+1} + g_{i+2}) / (2 dx^3), used for the
    gradient of the Laplacian in eq:F2."""
    return (-shift(g, -2) + 2.0 * shift(g, -1) - 2.0 * shift(g, 1) + shift(g, 2)) / (2.0 * dx ** 3)


def vlasov_force_ev2(n, p: Params):
    """eq:F2: F = 2 a dn/dx + kappa d3n/dx3 (1D), both derivatives by the
    5-point central stencils."""
    a = model.attraction_parameter(p.sigma, p.phi, p.gamma)
    kap = model.gradient_coefficient(p.sigma, p.phi, p.gamma)
    return 2.0 * a * central_gradient(n, p.dx) + kap * third_derivative(n, p.dx)


def vlasov_force(n, tb: Tables):
    p = tb.p
    if p.force_model == FORCE_EV1:
        Fx = vlasov_force_ev1(n, tb)
    elif p.force_model == FORCE_EV2:
        Fx = vlasov_force_ev2(n, p)
    else:
        Fx = np.zeros_like(n)
    return Fx + p.g_ext


# --- Hermite equilibrium ---

def equilibrium(n, u, T, tb: Tables):
    """E_k = sum_l M[k, l] a_l(n, u, T): the Hermite expansion (all orders
    l <= Q-1) of the 1D Maxwellian with density n, velocity u and
    temperature T.  Reading: the full expansion is used; it reproduces the
    Maxwellian moments exactly up to order Q-1."""
    a = hermite_moments_maxwellian(n, u, T, tb.p.Q)
    return tb.Meq @ a


# --- Shakhov model and J1 (reduced over p_y, p_z) ---

def shakhov(E, u, T, n, q, Pr, tb: Tables):
    """Reduced Shakhov distribution.

    f^S = f_MB [1 + (1 - Pr)/(P_i T) (xi^2/(5T) - 1) xi.q] integrated over
    (p_y, p_z) with weights 1 and (p_y^2+p_z^2)/2 gives, with
    theta = xi_x^2 / T and s = (1 - Pr) q / (5 n T^2),
        F^S = E [1 + s xi (theta - 3)]
        G^S = T E [1 + s xi (theta - 1)].
    """
    xi = tb.v[:, None] - u[None, :]
    th = xi ** 2 / T[None, :]
    s = ((1.0 - Pr) * q / (5.0 * n * T ** 2))[None, :]
    FS = E * (1.0 + s * xi * (th - 3.0))
    GS = T[None, :] * E * (1.0 + s * xi * (th - 1.0))
    return FS, GS


def j1_terms(E, u, T, n, chi, A, B, U, tb: Tables):
    """Reduced J1(f_MB, f_MB) (eq:J1) for a density varying along x only.

    With zeta = xi/sqrt(2T), A = d ln(rho^2 chi T)/dx, B = d ln T/dx,
    U = du/dx and theta = xi_x^2/T the (p_y, p_z) integrals give
        J1F = -b n chi E [xi (A + 0.3 (theta-3) B) + 0.6 (theta-1) U]
        J1G = -b n chi T E [xi (A + 0.3 (theta-1) B) + 0.2 (3 theta-1) U].
    """
    b = model.excluded_volume(tb.p.sigma)
    xi = tb.v[:, None] - u[None, :]
    th = xi ** 2 / T[None, :]
    pre = (-b * n * chi)[None, :]
    A, B, U = A[None, :], B[None, :], U[None, :]
    J1F = pre * E * (xi * (A + 0.3 * (th - 3.0) * B) + 0.6 * (th - 1.0) * U)
    J1G = pre * T[None, :] * E * (xi * (A + 0.3 * (th - 1.0) * B) + 0.2 * (3.0 * th - 1.0) * U)
    return J1F, J1G


# --- WENO-5 advection ---

def weno5_reconstruct(fm2, fm1, f0, fp1, fp2, eps):
    """Classical WENO-5 (Jiang-Shu) value at the right face of the centre
    cell from the five upwind-ordered values f_{i-2}..f_{i+2}."""
    q0 = (2.0 * fm2 - 7.0 * fm1 + 11.0 * f0) / 6.0
    q1 = (-fm1 + 5.0 * f0 + 2.0 * fp1) / 6.0
    q2 = (2.0 * f0 + 5.0 * fp1 - fp2) / 6.0
    b0 = 13.0 / 12.0 * (fm2 - 2.0 * fm1 + f0) ** 2 + 0.25 * (fm2 - 4.0 * fm1 + 3.0 * f0) ** 2
    b1 = 13.0 / 12.0 * (fm1 - 2.0 * f0 + fp1) ** 2 + 0.25 * (fm1 - fp1) ** 2
    b2 = 13.0 / 12.0 * (f0 - 2.0 * fp1 + fp2) ** 2 + 0.25 * (3.0 * f0 - 4.0 * fp1 + fp2) ** 2
    a0 = 0.1 / (eps + b0) ** 2
    a1 = 0.6 / (eps + b1) ** 2
    a2 = 0.3 / (eps + b2) ** 2
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2)


def weno5_advection(f, tb: Tables):
    """-p_k (fhat_{i+1/2} - fhat_{i-1/2}) / dx for every velocity row;
    upwind by the sign of p_k (Q even: no p = 0 node)."""
    eps = tb.p.weno_eps
    out = np.zeros_like(f)
    for k, pk in enumerate(tb.v):
        g = f[k]
        if pk > 0:
            fh = weno5_reconstruct(shift(g, -2), shift(g, -1), g, shift(g, 1), shift(g, 2), eps)
        else:
            # face i+1/2 seen from the right: mirror of the stencil
            fh = weno5_reconstruct(shift(g, 3), shift(g, 2), shift(g, 1), g, shift(g, -1), eps)
        out[k] = -pk * (fh - shift(fh, -1)) / tb.p.dx
    return out


# --- assembled right-hand side and time step ---

def node_fields(F, G, tb: Tables):
    """All per-node quantities the kinetic terms need at one stage."""
    p = tb.p
    n, u, T, q = moments(F, G, tb)
    if p.T_iso:
        T = np.full_like(T, p.T_iso)
    nbar = averaged_density(n, tb)
    chi = model.contact_value(nbar, p.sigma)
    Fx = vlasov_force(n, tb)
    nu = model.collision_rate(n, T, chi, p.sigma)
    Pr = model.prandtl(n, chi, p.sigma)
    X = n ** 2 * chi * T
    A = central_gradient(X, p.dx) / X
    B = central_gradient(T, p.dx) / T
    U = central_gradient(u, p.dx)
    return dict(n=n, u=u, T=T, q=q, nbar=nbar, chi=chi, Fx=Fx, nu=nu, Pr=Pr,
                X=X, A=A, B=B, U=U)


def rhs(F, G, tb: Tables):
    """L(F, G) of the semi-discrete system."""
    p = tb.p
    m = node_fields(F, G, tb)
    E = equilibrium(m["n"], m["u"], m["T"], tb)
    LF = np.zeros_like(F)
    LG = np.zeros_like(G)
    if p.term_mask & TERM_ADV:
        LF = LF + weno5_advection(F, tb)
        LG = LG + weno5_advection(G, tb)
    if p.term_mask & TERM_FORCE:
        LF = LF - m["Fx"][None, :] * (tb.Dp @ F)
        LG = LG - m["Fx"][None, :] * (tb.Dp @ G)
    if p.term_mask & TERM_J0:
        FS, GS = shakhov(E, m["u"], m["T"], m["n"], m["q"], m["Pr"], tb)
        LF = LF - m["nu"][None, :] * (F - FS)
        LG = LG - m["nu"][None, :] * (G - GS)
    if p.term_mask & TERM_J1:
        J1F, J1G = j1_terms(E, m["u"], m["T"], m["n"], m["chi"], m["A"], m["B"], m["U"], tb)
        LF = LF + J1F
        LG = LG + J1G
    return LF, LG


RK3_COEFFS = ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0))


def rk3_step(F, G, tb: Tables):
    """Third-order TVD Runge-Kutta (Shu-Osher):
    f1 = f^n + dt L(f^n); f2 = 3/4 f^n + 1/4 (f1 + dt L(f1));
    f^{n+1} = 1/3 f^n + 2/3 (f2 + dt L(f2))."""
    dt = tb.p.dt
    Fs, Gs = F, G
    for a, b in RK3_COEFFS:
        LF, LG = rhs(Fs, Gs, tb)
        Fs, Gs = a * F + b * (Fs + dt * LF), a * G + b * (Gs + dt * LG)
    return Fs, Gs


def run(F, G, tb: Tables, nsteps):
    for _ in range(nsteps):
        F, G = rk3_step(F, G, tb)
    return F, G


def initial_state(n, u, T, tb: Tables):
    """F = E(n, u, T), G = T E: the reduced Maxwellian of the given fields."""
    n = np.asarray(n)
    u = np.broadcast_to(np.asarray(u, dtype=np.result_type(n, u)), n.shape)
    T = np.broadcast_to(np.asarray(T, dtype=np.result_type(n, T)), n.shape)
    E = equilibrium(n, u, T, tb)
    return E, T[None, :] * E
