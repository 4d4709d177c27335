/*
 * evlb.h -- C ABI of the MI355X (gfx950) Enskog-Vlasov finite-difference
 * lattice Boltzmann (EV-FDLB) time step.
 *
 * Method: Busuioc & Sofonea, "Thermal Enskog-Vlasov Lattice Boltzmann model
 * with phase separation", arXiv:2503.15187.  The library advances the
 * reduced 1D distributions F(x, p), G(x, p) of a fluid homogeneous in y and
 * z (Sec. III) under the simplified Enskog-Vlasov equation (eq:enskog_approx
 * with the EV1 force eq:F1, or the EV2 force eq:F2), discretised on an
 * off-lattice full-range Gauss-Hermite velocity set, with WENO-5 advection,
 * 4th-order central gradients and TVD Runge-Kutta 3 in time (Sec. III,
 * numerical schemes paragraph).
 *
 * Conventions shared by every call
 *  - All floating point is IEEE double (FP64).
 *  - Pointers named d_* are DEVICE pointers (HIP global memory on the device
 *    current at evlb_init).  Pointers named h_* or documented as host are
 *    host memory.  The library allocates no device memory: the caller owns
 *    the state, the outputs and the workspace, and must keep the workspace
 *    alive and untouched while the context exists.
 *  - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued asynchronously on it; results are ready when the
 *    stream is synchronised.
 *  - Distribution layout: d_f[2][q][n_tot], structure of arrays, node index
 *    fastest.  Plane 0 holds F_k, plane 1 holds G_k; the velocity rows k are
 *    the Gauss-Hermite nodes in ascending order.  System s occupies nodes
 *    [off_s, off_s + nx[s]) with off_s = nx[0] + ... + nx[s-1]; each system
 *    is periodic on its own.
 *  - Node-field layout: d_n, d_u, d_T, d_q are [n_tot].
 *  - dim = 2 (a fluid homogeneous in z; the paper's 1D model extended along
 *    y, see evlb_params.dim): one periodic nx x ny system, n_tot = nx ny,
 *    q = 16 nodes per velocity component, node-major d_f[2][ny][nx][q][q]:
 *    d_f[d][y][x][k][l] is F (d = 0) or G (d = 1) at node (x, y) and
 *    velocity (p_x, p_y) = (p_k, p_l), the q^2 values of a node contiguous
 *    (whole cache lines per node and velocity row); F = int f dp_z,
 *    G = int p_z^2/2 f dp_z.  Node fields stay [n_tot] per component with
 *    node index y nx + x; vector node fields (u, q) are [2][n_tot] (x then y
 *    component).
 *  - Return value: EVLB_OK or a negative error code.  Argument errors are
 *    detected on the host before any device work is enqueued and leave all
 *    buffers untouched.  Device-detected errors (a non-positive or
 *    non-finite density or temperature produced by a step) are latched in
 *    the workspace and reported by evlb_status.
 *  - A context is bound to one device and is not thread-safe; calls that
 *    share a workspace must be ordered on one stream.
 */
#ifndef EVLB_H
#define EVLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EVLB_ABI_VERSION 4

enum {
  EVLB_OK = 0,
  EVLB_EINVAL = -1,       /* bad argument or parameter                      */
  EVLB_ECFL = -2,         /* dt * max|p_k| / dx above the stability limit   */
  EVLB_EWORKSPACE = -3,   /* workspace missing, too small or misaligned     */
  EVLB_EHIP = -4,         /* a HIP runtime call failed                      */
  EVLB_ENONFINITE = -5,   /* a step produced n <= 0, T <= 0 or NaN          */
  EVLB_EUNSUPPORTED = -6  /* valid but not built (e.g. quadrature order)    */
};

/* Self-consistent force model (Sec. II C, eq:ev_12). */
enum { EVLB_FORCE_EV1 = 0, EVLB_FORCE_EV2 = 1, EVLB_FORCE_NONE = 2 };

/* Right-hand-side terms; production runs use EVLB_TERM_ALL.  The others
 * exist to test one term at a time. */
enum {
  EVLB_TERM_ADV = 1,    /* -p dF/dx (WENO-5)                                */
  EVLB_TERM_FORCE = 2,  /* -F[n] dF/dp                                      */
  EVLB_TERM_J0 = 4,     /* -(chi/tau)(f - f^S), Shakhov                     */
  EVLB_TERM_J1 = 8,     /* J1(f_MB, f_MB), eq:J1                            */
  EVLB_TERM_ALL = 15
};

/* Launch strategy of evlb_step. */
enum {
  EVLB_EXEC_AUTO = 0,       /* persistent for small grids, else per stage   */
  EVLB_EXEC_PER_STAGE = 1,  /* one fused kernel per Runge-Kutta stage       */
  EVLB_EXEC_PERSISTENT = 2  /* one cooperative launch for all nsteps        */
};

typedef struct {
  int32_t abi_version;   /* must be EVLB_ABI_VERSION                         */
  int32_t dim;           /* 1, or 2 (the same model homogeneous in z only:
                            the z-integrated kernel of eq:force over a disc,
                            the averaged density of Sec. II A integrated
                            along z, Shakhov and J1 reduced over p_z).
                            dim 2 needs n_sys = 1, q = 16, gamma = 6, force
                            EV1 or none, r_cut/dx an integer <= 24,
                            sigma/dx <= 22, exec_mode AUTO or PER_STAGE,
                            tile_nodes 0, adjoint 0, and
                            dt 2 max|p_k| / dx <= 1                          */
  int32_t n_sys;         /* >= 1 independent periodic systems                */
  const int32_t* nx;     /* host [n_sys]: nodes per system, each >= 8        */
  int32_t q;             /* Gauss-Hermite order: 8, 16 or 24                 */
  double dx;             /* grid spacing; r_cut/dx an even integer, sigma/dx  
                            within 1e-3 of one (the averaging window)        */
  double dt;             /* time step                                        */
  double sigma;          /* hard-sphere diameter (eq:sutherland)             */
  double phi_sigma;      /* well depth of the attractive tail                */
  double gamma;          /* tail exponent (> 3; > 5 for EV2)                 */
  double r_cut;          /* truncation radius of the EV1 kernel (absolute)   */
  int32_t force_model;   /* EVLB_FORCE_*                                     */
  int32_t term_mask;     /* EVLB_TERM_* bits                                 */
  double weno_eps;       /* WENO-5 epsilon, 1e-6                             */
  double g_ext;          /* uniform external acceleration (tests), usually 0 */
  int32_t exec_mode;     /* EVLB_EXEC_*                                      */
  int32_t tile_nodes;    /* nodes per workgroup tile: 0 = auto, 16, 63 or 64 */
  int32_t adjoint;       /* 1: size the workspace for evlb_adjoint_step      */
  int32_t ny;            /* dim 2: nodes along y (>= 8); ignored for dim 1   */
  double T_iso;          /* > 0: isothermal run at this temperature, as in
                            the stationary-interface runs of Sec. III A
                            where T is kept constant: every kinetic term
                            (equilibrium, Shakhov, transport, J1) uses T_iso
                            instead of the moment temperature, so grad T = 0
                            and the energy is not conserved.  0: the thermal
                            model.  Not available with adjoint = 1.          */
  const double* T_iso_sys; /* NULL, or host [n_sys]: a fixed temperature per
                            system (>= 0, finite; 0 = thermal), overriding
                            T_iso, so that a sweep of the Sec. III A
                            stationary interfaces over T runs as one batch.
                            Copied by evlb_init.  dim 1 only; not available
                            with adjoint = 1 (EVLB_EUNSUPPORTED).  Adds
                            8 bytes per node to the workspace.              */
} evlb_params;

typedef struct evlb_ctx evlb_ctx; /* opaque, host memory */

/* Host only.  Checks a parameter set; EVLB_OK if evlb_init would accept it
 * (apart from the workspace).  No device call. */
int evlb_validate(const evlb_params* params);

/* Host only.  Bytes of device workspace evlb_init needs for these
 * parameters, or 0 if they are invalid.  The workspace must be 256-byte
 * aligned. */
size_t evlb_workspace_bytes(const evlb_params* params);

/* Builds the quadrature (roots of He_q, normalised Christoffel weights),
 * the Hermite equilibrium and momentum-derivative tables, the Simpson
 * weights of the averaged density (Sec. II A) and of the force (eq:F1),
 * enqueues their copies into d_workspace (and the clearing of the status
 * latch) on hip_stream, then synchronises hip_stream before returning (the
 * host staging buffers do not outlive the call), and returns a context in
 * *out.  d_workspace: device, >= evlb_workspace_bytes(params) bytes,
 * owned by the caller.  The context keeps a copy of params (and of nx). */
int evlb_init(const evlb_params* params, void* d_workspace, size_t ws_bytes,
              void* hip_stream, evlb_ctx** out);

/* Largest workspace evlb_init_noalloc serves (64 MiB: every dim-1 case up to
 * about 80 000 nodes, dim 2 up to about 90 x 90 nodes). */
#define EVLB_NOALLOC_MAX_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): evlb_init with
 * the library's own workspace, a static device array of
 * EVLB_NOALLOC_MAX_BYTES per device that the library holds until the
 * process ends, instead of a caller buffer.  Calls no hipMalloc or other
 * allocating routine.  Returns EVLB_EWORKSPACE if
 * evlb_workspace_bytes(params) exceeds EVLB_NOALLOC_MAX_BYTES, EVLB_EHIP if
 * the array's device address cannot be obtained.  Every context made this
 * way on one device shares that device's array: a new one re-initialises it
 * and invalidates the previous one (its later calls give undefined
 * results), and calls of such contexts that overlap on one device race.
 * The context is released with evlb_destroy as any other. */
int evlb_init_noalloc(const evlb_params* params, void* hip_stream, evlb_ctx** out);

/* Writes the reduced Maxwellian of the given node fields into d_f:
 * F_k = E_k(n, u, T) (Hermite expansion to order q-1), G_k = T E_k.
 * d_n, d_u, d_T: device [n_tot], read only.  d_f: device [2][q][n_tot].
 * dim 2: d_u is [2][n_tot], d_f is node-major [2][ny][nx][q][q] (see the
 * layout notes above), F_kl = n e_k(u_x) e_l(u_y) (the product of the
 * unit-density expansions), G_kl = T/2 F_kl. */
int evlb_set_equilibrium(evlb_ctx* ctx, const double* d_n, const double* d_u,
                         const double* d_T, double* d_f, void* hip_stream);

/* Advances d_f (device [2][q][n_tot], in/out) by nsteps >= 0 TVD-RK3 steps
 * of size dt.  Every stage re-evaluates the moments, the averaged density
 * and contact value (eq:carnstar), the Vlasov force (eq:F1 / eq:F2), the
 * transport coefficients (eq:viscosity, eq:tau, eq:prandtl), the Hermite
 * equilibrium, the Shakhov term, J1 (eq:J1), the momentum derivative and
 * the WENO-5 flux.  Uses the workspace for stage buffers. */
int evlb_step(evlb_ctx* ctx, double* d_f, int32_t nsteps, void* hip_stream);

/* Right-hand side L(f) of the semi-discrete system at one state:
 * d_L[2][q][n_tot] = dF/dt, dG/dt (device).  d_f is read only. */
int evlb_rhs(evlb_ctx* ctx, const double* d_f, double* d_L, void* hip_stream);

/* Moments of d_f (Sec. II B): n = sum F, n u = sum p F,
 * 3/2 n T = sum (xi^2/2 F + G), q = sum xi (xi^2/2 F + G), xi = p - u
 * (T is the moment temperature also in isothermal runs).
 * Outputs device [n_tot]; d_q may be NULL.  dim 2: xi is the in-plane
 * peculiar velocity and d_u, d_q are [2][n_tot]. */
int evlb_moments(evlb_ctx* ctx, const double* d_f, double* d_n, double* d_u,
                 double* d_T, double* d_q, void* hip_stream);

/* Discrete adjoint of one evlb_step step (rows of the method as above, the
 * TVD-RK3 scheme transposed stage by stage).  Given d_lam_np1 = dL/df^{n+1}
 * for the state after the step and d_f_n = the state before it, writes
 * d_lam_n = dL/df^n through the step, and ADDS to d_dparams[0..1] the
 * explicit derivatives dL/dphi_sigma and dL/dsigma of this step (the node
 * window of the averaged density stays fixed; the kernel switches branch at
 * |x' - x| >= sigma, so the sigma derivative is the one-sided derivative from
 * below where a node sits on sigma).  All pointers are device: d_f_n,
 * d_lam_np1, d_lam_n [2][q][n_tot], d_dparams [2].  d_lam_n must not alias
 * d_lam_np1 or d_f_n.  Requires params.adjoint = 1 and force model EV1 or
 * none (EVLB_EINVAL otherwise); dim 2 returns EVLB_EUNSUPPORTED, as do the
 * record and equilibrium-adjoint calls below.  The stage buffers of the
 * workspace are overwritten. */
int evlb_adjoint_step(evlb_ctx* ctx, const double* d_f_n, const double* d_lam_np1,
                      double* d_lam_n, double* d_dparams, void* hip_stream);

/* Number of doubles of one step record of evlb_step_record: the state, the
 * two inner Runge-Kutta stage states and the moments of the three,
 * 3 * 2 * q * n_tot + 12 * n_tot. */
int64_t evlb_record_doubles(const evlb_ctx* ctx);

/* Advances d_f0 (device [2][q][n_tot], read only) by nsteps steps, keeping
 * every step: d_rec (device, (nsteps + 1) * evlb_record_doubles) receives
 * record j = {f^j, f1^j, f2^j, moments of the three} for j < nsteps, and
 * record nsteps starts with f^nsteps (its stages are left unwritten). */
int evlb_step_record(evlb_ctx* ctx, const double* d_f0, int32_t nsteps, double* d_rec,
                     void* hip_stream);

/* Runs evlb_adjoint_step backwards over a record of nsteps steps without
 * recomputing stages.  d_lam (device [2][q][n_tot]) holds dL/df^nsteps on
 * entry and dL/df^0 on return.  Optional per-step linear observable: with
 * d_obs (device [2][q][n_tot]) and d_w (device [nsteps]), the loss is taken
 * to contain sum_j w[j] <d_obs, f^{j+1}>, i.e. dL/df^{j+1} += w[j] d_obs
 * before step j is transposed (both NULL: none).  d_dparams as for
 * evlb_adjoint_step. */
int evlb_adjoint_record(evlb_ctx* ctx, const double* d_rec, int32_t nsteps, double* d_lam,
                        const double* d_obs, const double* d_w, double* d_dparams,
                        void* hip_stream);

/* Adjoint of evlb_set_equilibrium: for lam = dL/df (device [2][q][n_tot])
 * writes dL/dn, dL/du, dL/dT (device [n_tot] each) of the state
 * F = E(n, u, T), G = T E. */
int evlb_equilibrium_adjoint(evlb_ctx* ctx, const double* d_n, const double* d_u,
                             const double* d_T, const double* d_lam, double* d_nbar,
                             double* d_ubar, double* d_Tbar, void* hip_stream);

/* Enqueues a copy of the latched device status to the host (and, when
 * clear != 0, its clearing) on hip_stream, synchronises hip_stream and
 * reports it: EVLB_OK or EVLB_ENONFINITE. */
int evlb_status(evlb_ctx* ctx, void* hip_stream, int32_t clear);

/* Node count n_tot and quadrature nodes (host copy, length q) of a context. */
int evlb_info(const evlb_ctx* ctx, int64_t* n_tot, double* h_velocities);

/* Releases the host context (not the caller's device memory). */
void evlb_destroy(evlb_ctx* ctx);

/* Static description of an error code. */
const char* evlb_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* EVLB_H */
