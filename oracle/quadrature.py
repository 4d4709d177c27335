"""Full-range Gauss-Hermite velocity set (test infrastructure, see package doc).

The paper discretises momentum space with off-lattice full-range
Gauss-Hermite quadratures of order Q_x = 16 (Sec. III, numerical schemes
paragraph; Sec. I cites the FDLB literature for the construction).  The
reduced distributions F, G are represented by their values f_k at the
quadrature nodes p_k, scaled so that plain sums over k are integrals:

    sum_k f_k g(p_k)  ==  integral f(p) g(p) dp    (exact for polynomial g
                                                    of degree <= 2Q-1 times
                                                    the Gaussian weight)

Reading (paper silent): nodes are the roots of the probabilists' Hermite
polynomial He_Q (weight exp(-p^2/2)), not rescaled by the local
temperature, and the weights are normalised to sum to one.
"""
import math

import numpy as np


def hermite_table(x, lmax):
    """He_0(x) .. He_lmax(x) by the three-term recurrence
    He_{l+1} = x He_l - l He_{l-1}.  Returns shape (lmax+1,) + x.shape."""
    x = np.asarray(x)
    H = np.zeros((lmax + 1,) + x.shape, dtype=np.result_type(x, np.float64))
    H[0] = 1.0
    if lmax >= 1:
        H[1] = x
    for l in range(1, lmax):
        H[l + 1] = x * H[l] - l * H[l - 1]
    return H


def gauss_hermite(Q):
    """Nodes p_k (ascending) and normalised weights w_k of the Q-point
    Gauss rule for the weight exp(-p^2/2)/sqrt(2 pi).

    Nodes: eigenvalues of the symmetric Jacobi matrix of the monic He
    recurrence (off-diagonal sqrt(l)), polished by Newton steps on He_Q.
    Weights: Christoffel numbers w_k = Q! / (Q He_{Q-1}(p_k))^2, which sum
    to one for this normalisation.
    """
    if Q < 2:
        raise ValueError("Q must be >= 2")
    off = np.sqrt(np.arange(1, Q, dtype=np.float64))
    J = np.diag(off, 1) + np.diag(off, -1)
    x = np.linalg.eigvalsh(J)
    for _ in range(4):
        H = hermite_table(x, Q)
        x = x - H[Q] / (Q * H[Q - 1])
    # the rule is symmetric about p = 0; enforce it exactly
    x = 0.5 * (x - x[::-1])
    H = hermite_table(x, Q)
    w = math.factorial(Q) / (Q * H[Q - 1]) ** 2
    w = 0.5 * (w + w[::-1])
    return x, w


def equilibrium_matrix(p, w):
    """M[k, l] = w_k He_l(p_k) / l!  for l = 0..Q-1.

    The Hermite expansion of a distribution with Hermite moments
    a_l = integral He_l(p) f(p) dp is f_k = sum_l M[k, l] a_l.
    """
    Q = len(p)
    H = hermite_table(p, Q - 1)
    fact = np.array([math.factorial(l) for l in range(Q)], dtype=np.float64)
    return (w[:, None] * H.T) / fact[None, :]


def momentum_derivative_matrix(p, w):
    """Dp[k, k'] such that (Dp f)_k represents d f / d p at node k.

    f is projected on Hermite polynomials, b_l = sum_k' He_l(p_k') f_k',
    f(p) ~ omega(p) sum_l He_l(p) b_l / l!, and the derivative of
    omega He_l is -omega He_{l+1}, so

        (Dp f)_k = - w_k sum_{l=0}^{Q-2} He_{l+1}(p_k) b_l / l!

    (the l = Q-1 term vanishes at the nodes because He_Q(p_k) = 0).
    """
    Q = len(p)
    H = hermite_table(p, Q)
    D = np.zeros((Q, Q))
    for l in range(Q - 1):
        D -= np.outer(w * H[l + 1], H[l]) / math.factorial(l)
    return D


def hermite_moments_maxwellian(n, u, T, Q):
    """a_l = integral He_l(p) f_MB(p) dp, l = 0..Q-1, for the 1D Maxwellian
    of density n, velocity u, temperature T (m = k_B = 1):
    a_0 = n, a_1 = n u, a_{l+1} = u a_l + l (T - 1) a_{l-1}."""
    n = np.asarray(n)
    a = np.zeros((Q,) + n.shape, dtype=np.result_type(n, u, T, np.float64))
    a[0] = n
    if Q > 1:
        a[1] = n * u
    for l in range(1, Q - 1):
        a[l + 1] = u * a[l] + l * (T - 1.0) * a[l - 1]
    return a
