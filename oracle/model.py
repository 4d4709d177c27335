"""Model ingredients of the EV-FDLB method (test infrastructure).

Units: m = k_B = 1; lengths in sigma-units when sigma = 1; k_B T_ref equal
to the well depth phi_sigma (this reading reproduces the paper's critical
temperature, see critical_point).  Every routine is generic in dtype
(float64 / complex128); branches are taken on real parts so that a complex
perturbation of sigma or phi_sigma follows one branch.
"""
import math
from dataclasses import dataclass, field

import numpy as np

TERM_ADV, TERM_FORCE, TERM_J0, TERM_J1 = 1, 2, 4, 8
TERM_ALL = 15
FORCE_EV1, FORCE_EV2, FORCE_NONE = 0, 1, 2


@dataclass
class Params:
    """Parameters of one 1D system (the paper's statement of the problem:
    sigma, phi_sigma, gamma of the Sutherland potential; the numerical
    parameters dt, dx and quadrature order Q).

    r_cut: absolute truncation radius of the attractive kernel (the paper
    gives none; 5 sigma is used).  term_mask / g_ext are test switches:
    g_ext is a uniform external force added to the Vlasov force.
    T_iso > 0 selects the isothermal runs of Sec. III A, where the fluid
    temperature is kept constant: the node temperature every kinetic term
    sees (equilibrium, Shakhov, transport, J1) is T_iso instead of the
    moment of f, so grad T = 0.  T_iso = 0 is the thermal model.
    """
    Q: int
    dx: float
    dt: float
    sigma: complex = 1.0
    phi: complex = 1.0
    gamma: float = 6.0
    r_cut: float = 5.0
    force_model: int = FORCE_EV1
    term_mask: int = TERM_ALL
    weno_eps: float = 1e-6
    g_ext: float = 0.0
    sigma_ref: float = field(default=None)  # fixes the node windows
    T_iso: float = 0.0

    def __post_init__(self):
        if self.sigma_ref is None:
            self.sigma_ref = float(np.real(self.sigma))


# ---------------------------------------------------------------------------
# contact value (eq:carnstar) and Fischer-Methfessel average
# ---------------------------------------------------------------------------

def packing_fraction(n, sigma):
    """eta = pi sigma^3 n / 6 (eq:carnstar)."""
    return np.pi * sigma ** 3 * n / 6.0


def excluded_volume(sigma):
    """b = 2 pi sigma^3 / 3 (eq:carnstar)."""
    return 2.0 * np.pi * sigma ** 3 / 3.0


def contact_value(nbar, sigma):
    """chi_SET from the Carnahan-Starling equation of state,
    chi = (2 - eta) / (2 (1 - eta)^3), evaluated at the averaged density
    (eq:carnstar, second form)."""
    eta = packing_fraction(nbar, sigma)
    return (2.0 - eta) / (2.0 * (1.0 - eta) ** 3)


def compressibility_factor(n, sigma):
    """Carnahan-Starling Z = (1 + eta + eta^2 - eta^3) / (1 - eta)^3, the
    hard-sphere part of eq:EOSS."""
    eta = packing_fraction(n, sigma)
    return (1.0 + eta + eta ** 2 - eta ** 3) / (1.0 - eta) ** 3


def simpson_pattern(M2):
    """Composite Simpson 1/3 weights (1,4,2,4,...,2,4,1)/3 over M2 (even)
    equal intervals; returns M2 + 1 values."""
    if M2 % 2:
        raise ValueError("Simpson's rule needs an even number of intervals")
    s = np.ones(M2 + 1)
    s[1:M2:2] = 4.0
    s[2:M2:2] = 2.0
    s[0] = s[M2] = 1.0
    return s / 3.0


def averaging_weights(p: Params):
    """Weights s_j, j = -Ms..Ms, of the averaged density
    nbar_i = sum_j s_j n_{i+j}.

    The Fischer-Methfessel average (Sec. II A) over a ball of radius sigma,
    for a density that depends on x only, reduces to
        nbar(x) = 3/(4 sigma^3) * integral_{-sigma}^{sigma} (sigma^2 - s^2) n(x+s) ds
    (the ball's cross-section at offset s is pi (sigma^2 - s^2)).
    Reading: the integral is taken with the same composite Simpson rule the
    paper names for the force, on the grid nodes, so sigma/dx must be even.
    The node window is fixed by sigma_ref; the weights follow sigma.
    """
    Ms = int(round(p.sigma_ref / p.dx))
    if abs(Ms * p.dx - p.sigma_ref) > 1e-12 * p.sigma_ref or Ms % 2:
        raise ValueError("sigma/dx must be an even integer")
    s = np.arange(-Ms, Ms + 1) * p.dx
    sig = p.sigma
    return 3.0 / (4.0 * sig ** 3) * (sig ** 2 - s ** 2) * p.dx * simpson_pattern(2 * Ms)


def force_kernel_1d(s, p: Params):
    """Planar (y,z-integrated) kernel of the Vlasov force, eq:F1:
        K(s) = 2 pi phi_sigma * s                      |s| <  sigma
        K(s) = 2 pi phi_sigma * sigma^gamma s/|s|^gamma  |s| >= sigma
    so that F(x) = integral K(x' - x) n(x') dx'."""
    s = np.asarray(s, dtype=np.float64)
    out = np.empty(s.shape, dtype=np.result_type(p.sigma, p.phi, np.float64))
    inner = np.abs(s) < np.real(p.sigma)
    out[inner] = 2.0 * np.pi * p.phi * s[inner]
    so = s[~inner]
    out[~inner] = 2.0 * np.pi * p.phi * p.sigma ** p.gamma * so / np.abs(so) ** p.gamma
    return out


def force_weights(p: Params):
    """c_j, j = 1..MF, of F_i = sum_j c_j (n_{i+j} - n_{i-j}).

    eq:F1 integrated with the composite Simpson 1/3 rule over the window
    |x' - x| <= r_cut (reading: the paper states no cutoff; the tail beyond
    r_cut is dropped) on the grid nodes x' = x + j dx.  K is odd, so the
    j and -j terms pair up.  With sigma/dx even the kink of K at |s| = sigma
    falls on a Simpson panel boundary.
    """
    MF = int(round(p.r_cut / p.dx))
    if abs(MF * p.dx - p.r_cut) > 1e-12 * p.r_cut or MF % 2:
        raise ValueError("r_cut/dx must be an even integer")
    j = np.arange(-MF, MF + 1)
    c = force_kernel_1d(j * p.dx, p) * p.dx * simpson_pattern(2 * MF)
    return c[MF + 1:]


def attraction_parameter_discrete(p: Params):
    """a_disc = sum_j c_j (j dx): the long-wave limit F -> 2 a_disc dn/dx of
    the discrete force (the continuum value is eq:F2's a)."""
    c = force_weights(p)
    j = np.arange(1, len(c) + 1)
    return np.sum(c * j * p.dx)


def attraction_parameter(sigma=1.0, phi=1.0, gamma=6.0):
    """a = (2 pi sigma^3 / 3) phi_sigma gamma / (gamma - 3) (eq:F2)."""
    return 2.0 * np.pi * sigma ** 3 / 3.0 * phi * gamma / (gamma - 3.0)


def gradient_coefficient(sigma=1.0, phi=1.0, gamma=6.0):
    """kappa = (2 pi sigma^5 / 15) phi_sigma gamma / (gamma - 5) (eq:F2)."""
    return 2.0 * np.pi * sigma ** 5 / 15.0 * phi * gamma / (gamma - 5.0)


# ---------------------------------------------------------------------------
# transport (eq:viscosity, eq:tau, eq:prandtl)
# ---------------------------------------------------------------------------

def viscosity(n, T, chi, sigma):
    """Enskog shear viscosity mu = mu0 [1/chi + 4/5 b rho + 4/25 (1+12/pi)
    (b rho)^2 chi], mu0 = 5/(16 sigma^2) sqrt(T/pi); rho = m n = n."""
    b = excluded_volume(sigma)
    mu0 = 5.0 / (16.0 * sigma ** 2) * np.sqrt(T / np.pi)
    brho = b * n
    return mu0 * (1.0 / chi + 0.8 * brho + 0.16 * (1.0 + 12.0 / np.pi) * brho ** 2 * chi)


def conductivity(n, T, chi, sigma):
    """Enskog thermal conductivity lambda = lambda0 [1/chi + 6/5 b rho +
    9/25 (1 + 32/(9 pi)) (b rho)^2 chi], lambda0 = 75/(64 sigma^2)
    sqrt(T/pi).  Not used by the step; used to check the Prandtl number."""
    b = excluded_volume(sigma)
    lam0 = 75.0 / (64.0 * sigma ** 2) * np.sqrt(T / np.pi)
    brho = b * n
    return lam0 * (1.0 / chi + 1.2 * brho + 0.36 * (1.0 + 32.0 / (9.0 * np.pi)) * brho ** 2 * chi)


def relaxation_time(n, T, chi, sigma):
    """tau = mu / (P_i (1 + 2/5 b rho chi)), P_i = n T (eq:tau)."""
    b = excluded_volume(sigma)
    return viscosity(n, T, chi, sigma) / (n * T * (1.0 + 0.4 * b * n * chi))


def collision_rate(n, T, chi, sigma):
    """nu = chi / tau, the rate of the Shakhov term J0 = -(chi/tau)(f - f^S).
    Reading: chi multiplies 1/tau literally, as written in the paper."""
    return chi / relaxation_time(n, T, chi, sigma)


def prandtl(n, chi, sigma):
    """eq:prandtl with y = b rho chi."""
    y = excluded_volume(sigma) * n * chi
    return (2.0 / 3.0) * (1.0 + 0.6 * y) / (1.0 + 0.4 * y) * \
        (1.0 + 0.8 * y + 0.16 * (1.0 + 12.0 / np.pi) * y ** 2) / \
        (1.0 + 1.2 * y + 0.36 * (1.0 + 32.0 / (9.0 * np.pi)) * y ** 2)


# ---------------------------------------------------------------------------
# equation of state (eq:EOSS), critical point, Maxwell construction
# ---------------------------------------------------------------------------

def pressure(n, T, a, sigma=1.0):
    """P = n T (1 + eta + eta^2 - eta^3)/(1 - eta)^3 - a n^2 (eq:EOSS)."""
    return n * T * compressibility_factor(n, sigma) - a * n ** 2


def chemical_potential(n, T, a, sigma=1.0):
    """Chemical potential of the EOS up to a function of T alone:
    T ln n + T (8 eta - 9 eta^2 + 3 eta^3)/(1 - eta)^3 - 2 a n.
    (Carnahan-Starling excess chemical potential plus the mean-field term;
    d mu / dn = (1/n) dP/dn holds, checked in the tests.)"""
    eta = packing_fraction(n, sigma)
    return T * np.log(n) + T * (8 * eta - 9 * eta ** 2 + 3 * eta ** 3) / (1 - eta) ** 3 - 2 * a * n


def _dP_dn(n, T, a, sigma=1.0):
    eta = packing_fraction(n, sigma)
    return T * (1 + 4 * eta + 4 * eta ** 2 - 4 * eta ** 3 + eta ** 4) / (1 - eta) ** 4 - 2 * a * n


def critical_point(a, sigma=1.0):
    """(n_c, T_c, P_c) where dP/dn = d2P/dn2 = 0 for eq:EOSS.

    With g1(eta) = d(nZ)/dn and g2 = d2(nZ)/dn2 the conditions are
    T g1 = 2 a n and T g2 = 2 a, i.e. g1/g2 = n, solved for eta by
    bisection, then T_c = 2 a / g2."""
    c = np.pi * sigma ** 3 / 6.0

    def g1(e):
        return (1 + 4 * e + 4 * e ** 2 - 4 * e ** 3 + e ** 4) / (1 - e) ** 4

    def g2(e):
        return c * (8 + 20 * e - 4 * e ** 2) / (1 - e) ** 5

    def h(e):
        return g1(e) / g2(e) - e / c

    lo, hi = 1e-6, 0.5
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if h(lo) * h(mid) <= 0:
            hi = mid
        else:
            lo = mid
    eta = 0.5 * (lo + hi)
    n = eta / c
    T = 2 * a / g2(eta)
    return n, T, pressure(n, T, a, sigma)


def spinodal(T, a, sigma=1.0):
    """Densities where dP/dn = 0 at temperature T < T_c (bisection on each
    side of the critical density)."""
    n_c, T_c, _ = critical_point(a, sigma)
    if T >= T_c:
        raise ValueError("T must be below T_c")

    def bis(lo, hi):
        flo = _dP_dn(lo, T, a, sigma)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            fm = _dP_dn(mid, T, a, sigma)
            if flo * fm <= 0:
                hi = mid
            else:
                lo, flo = mid, fm
        return 0.5 * (lo + hi)

    n_max = 6.0 / (np.pi * sigma ** 3)
    return bis(1e-12, n_c), bis(n_c, 0.999 * n_max)


def maxwell_construction(T, a, sigma=1.0):
    """Coexisting vapour and liquid densities (n_v, n_l) at temperature T:
    equal pressure and equal chemical potential, solved by Newton's method
    in (n_v, n_l) started outside the spinodal interval."""
    sv, sl = spinodal(T, a, sigma)
    nv, nl = 0.5 * sv, min(sl * 1.5, 0.95 * 6.0 / np.pi / sigma ** 3)
    for _ in range(200):
        Pv, Pl = pressure(nv, T, a, sigma), pressure(nl, T, a, sigma)
        mv, ml = chemical_potential(nv, T, a, sigma), chemical_potential(nl, T, a, sigma)
        r = np.array([Pl - Pv, ml - mv])
        if np.max(np.abs(r)) < 1e-15:
            break
        J = np.array([[-_dP_dn(nv, T, a, sigma), _dP_dn(nl, T, a, sigma)],
                      [-_dP_dn(nv, T, a, sigma) / nv, _dP_dn(nl, T, a, sigma) / nl]])
        d = np.linalg.solve(J, -r)
        # damped step keeping the two branches on their sides
        t = 1.0
        for _ in range(60):
            nv2, nl2 = nv + t * d[0], nl + t * d[1]
            if 0 < nv2 < sv and sl < nl2 < 6.0 / np.pi / sigma ** 3:
                break
            t *= 0.5
        nv, nl = nv2, nl2
    return nv, nl
