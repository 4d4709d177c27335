"""Seeded synthetic inputs for the EV-FDLB step.

This module generates initial fields (density, velocity, temperature) and
parameter sets with the shapes and value distributions of the paper's
workloads (Sec. III B phase separation from a perturbed uniform state,
Sec. III C liquid-slab evaporation with the tanh interfaces of eq:tan).
It holds none of the method's arithmetic: derived constants (temperatures,
coexistence densities, time steps) are read from constants.json, which a
committed script computes with the CPU oracle.  Both the oracle-side tests
and the HIP-side callers take their inputs from here.

Random numbers: numpy PCG64 (numpy.random.default_rng) with the seeds
recorded in constants.json.
"""
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


def constants():
    with open(os.path.join(_HERE, "constants.json")) as fh:
        return json.load(fh)


def grid(nx, dx):
    """Node positions x_i = (i - nx/2) dx of the periodic box [-L/2, L/2)."""
    return (np.arange(nx) - nx // 2) * dx


def tanh_slab(x, n_l, n_v, x0, width):
    """eq:tan: liquid slab of half-width x0 at density n_l surrounded by
    vapour at n_v/2, joined by tanh interfaces of the given width."""
    return n_l + (n_v - 2.0 * n_l) / 4.0 * (1.0 + np.tanh((np.abs(x) - x0) / width))


def uniform_noise(rng, n0, amp, size):
    """n0 (1 + amp (2U - 1)), U ~ uniform[0, 1)."""
    return n0 * (1.0 + amp * (2.0 * rng.random(size) - 1.0))


def phase_separation_1d(nx=None, seed=None):
    """Uniform fluid inside the spinodal with seeded +-1% uniform noise,
    at rest, uniform temperature.  Returns (params dict, n, u, T)."""
    c = dict(constants()["phase_separation_1d"])
    if nx is not None:
        c["nx"] = nx
    rng = np.random.default_rng(c["seed"] if seed is None else seed)
    n = uniform_noise(rng, c["n0"], c["noise"], c["nx"])
    return c, n, np.zeros(c["nx"]), np.full(c["nx"], c["T"])


def phase_separation_2d(nx=None, ny=None, seed=None):
    """2D uniform fluid inside the spinodal with seeded Gaussian noise,
    n0 (1 + amp N(0, 1)), at rest, uniform temperature.  Fields have shape
    (ny, nx).  Returns (params dict, n, ux, uy, T)."""
    c = dict(constants()["phase_separation_2d"])
    if nx is not None:
        c["nx"] = nx
    if ny is not None:
        c["ny"] = ny
    rng = np.random.default_rng(c["seed"] if seed is None else seed)
    shp = (c["ny"], c["nx"])
    n = c["n0"] * (1.0 + c["noise"] * rng.standard_normal(shp))
    z = np.zeros(shp)
    return c, n, z, z.copy(), np.full(shp, c["T"])


def paper_sec3b():
    """The four phase-separation runs of Sec. III B (eq:rho_init_takata):
    n = A (1 + omega cos(2 pi x / L)) on [-L/2, L/2), L = 100 sigma, at rest,
    uniform T_i, A = (n_l + n_v)/2 at T_i.  Returns (params dict, list of
    (n, u, T))."""
    c = dict(constants()["paper_sec3b_phase_separation"])
    x = grid(c["nx"], c["dx"])
    systems = []
    for (T, omega), A in zip(c["pairs"], c["A"]):
        n = A * (1.0 + omega * np.cos(2.0 * np.pi * x / c["L"]))
        systems.append((n, np.zeros(c["nx"]), np.full(c["nx"], T)))
    return c, systems


def paper_sec3c():
    """The four evaporation runs of Sec. III C: liquid slab (eq:tan) with
    interfaces at +-25 sigma in [-200 sigma, 200 sigma), vapour at n_v/2,
    at rest, uniform T_i.  Returns (params dict, list of (n, u, T))."""
    c = dict(constants()["paper_sec3c_evaporation"])
    x = grid(c["nx"], c["dx"])
    systems = []
    for T, nl, nv in zip(c["T"], c["n_l"], c["n_v"]):
        n = tanh_slab(x, nl, nv, c["x0"], c["width"])
        systems.append((n, np.zeros(c["nx"]), np.full(c["nx"], T)))
    return c, systems


def slab_1d(name="slab_evaporation_1d", nx=None, dx=None):
    """Liquid slab (eq:tan) centred in the periodic box, at rest, uniform
    temperature.  nx/dx may be overridden for reduced-size cases (the slab
    geometry is kept in sigma units).  Returns (params dict, n, u, T)."""
    c = dict(constants()[name])
    if nx is not None:
        c["nx"] = nx
    if dx is not None:
        c["dx"] = dx
    x = grid(c["nx"], c["dx"])
    n = tanh_slab(x, c["n_l"], c["n_v"], c["x0"], c["width"])
    return c, n, np.zeros(c["nx"]), np.full(c["nx"], c["T"])


def batched_sweep_1d(n_sys=None, seed=None, nx_max=None):
    """Independent periodic systems with log-uniform lengths, uniform
    T/T_c and mean densities, +-1% noise.  Returns (params dict, list of
    (n, u, T) per system)."""
    c = dict(constants()["batched_sweep_1d"])
    if n_sys is not None:
        c["n_sys"] = n_sys
    if nx_max is not None:
        c["nx_max"] = nx_max
    rng = np.random.default_rng(c["seed"] if seed is None else seed)
    lo, hi = np.log(c["nx_min"]), np.log(c["nx_max"])
    nxs = np.rint(np.exp(rng.uniform(lo, hi, c["n_sys"]))).astype(np.int64)
    tr = rng.uniform(c["t_over_tc"][0], c["t_over_tc"][1], c["n_sys"])
    n0 = rng.uniform(c["n0"][0], c["n0"][1], c["n_sys"])
    systems = []
    for i in range(c["n_sys"]):
        n = uniform_noise(rng, n0[i], c["noise"], int(nxs[i]))
        systems.append((n, np.zeros(int(nxs[i])), np.full(int(nxs[i]), tr[i] * c["Tc_disc"])))
    c["nx_list"] = [int(v) for v in nxs]
    return c, systems


def adjoint_target(c, n_init, seed=None):
    """Seeded target profile n* = n_init (1 + amp sum_m (a_m cos + b_m sin)
    (2 pi m x / L) / sqrt(M)), a, b ~ N(0, 1), for the misfit part of the
    gradient-check loss."""
    rng = np.random.default_rng(c["target_seed"] if seed is None else seed)
    M = c["target_modes"]
    a = rng.standard_normal(M)
    b = rng.standard_normal(M)
    L = c["nx"] * c["dx"]
    x = grid(c["nx"], c["dx"])
    pert = np.zeros_like(x)
    for m in range(1, M + 1):
        pert += a[m - 1] * np.cos(2 * np.pi * m * x / L) + b[m - 1] * np.sin(2 * np.pi * m * x / L)
    return n_init * (1.0 + c["target_amp"] * pert / np.sqrt(M))
