/* lbm.h -- C ABI of the MI355X (gfx950) collide-and-stream library.
 *
 * The library advances the per-field, exact-flux-equilibrium BGK lattice
 * Boltzmann scheme of Kummerlaender, Bukreev & Krause ("Automated Derivation
 * of Lattice Boltzmann Methods for Systems of Conservation Laws") on a
 * periodic grid:
 *
 *   Q_k        = Q0_k + sum_i f*_{k,i}                          eq. (moments),
 *                                                               Sec. 2.5.2 shift
 *   f*eq_{k,i} = w_i [ dQ_k + (dt/dx)/cs^2  c_i . (Phi_k(Q) - Phi_k(Q0)) ]
 *                                                               eq. (feq), shifted
 *   f*_{k,i}(x + c_i, t + dt) = f*_{k,i} - omega_k (f*_{k,i} - f*eq_{k,i})
 *                               + dt w_i S_k(x, t + dt/2)       eq. (lbe_update)
 *
 * with one population set per conserved field and per gradient tracker
 * (Sec. 2.1.1), conserved fields colliding at omega = 1/tau and trackers at
 * 1/(g_tau + 1) with tau_grad = g_tau dt (supplement, numerical
 * configuration).  Every step runs in hand-written HIP kernels; there is no
 * CPU path.
 *
 * Conventions
 *  - Every device pointer is memory the caller owns (e.g. a torch tensor);
 *    the library never allocates or frees device memory.
 *  - A field array is [K][nz][ny][nx], x fastest.  A population array is
 *    tile-blocked: the nx*ny cells of each z-slab, in-plane index
 *    yx = y nx + x, are cut into tiles of 64 consecutive cells, the last
 *    tile of a slab padded to 64, and a tile holds all K*Q populations of
 *    its cells, [nz][tiles][K][Q][64]: population (k, i) of cell (x, y, z)
 *    is element ((z T + yx / 64) K Q + k Q + i) 64 + yx % 64, with
 *    T = ceil(nx ny / 64) tiles per slab.  A wavefront's 64 cells of one
 *    population are one contiguous run and all its populations one block.
 *    Padding elements are never read.
 *  - Population order: D2Q5 = rest, +x, +y, -x, -y; D2Q9 = D2Q5 then
 *    (+1,+1), (-1,+1), (-1,-1), (+1,-1); D3Q7 = rest, +x, -x, +y, -y, +z, -z.
 *  - Calls are asynchronous on the bound HIP stream unless they return host
 *    data.  A handle is not thread-safe.  Status codes are below; the text of
 *    the last error is available from lbm_last_error.
 *  - Storage precision: LBM_F64 stores and computes in double; LBM_F32
 *    stores and computes in float; LBM_F16 stores the shifted populations in
 *    IEEE binary16 scaled by a per-field power of two and computes in float;
 *    LBM_F16NE keeps each cell's moment deviations in float and stores in
 *    binary16 only each population's deviation from that cell's own
 *    equilibrium (2D systems; the receiving cell rebuilds the population from
 *    the sender's moments).  Reductions accumulate in double in every case.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_state lbm_state;

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,        /* bad argument, unknown name, wrong order of calls */
    LBM_ENOTBOUND = -2,     /* device buffers not bound yet                      */
    LBM_EHIP = -3,          /* a HIP runtime call failed                         */
    LBM_ESUBCHAR = -4,      /* initial state violates the sub-characteristic bound */
    LBM_ENONFINITE = -5     /* non-finite populations detected                   */
};

enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16 = 2, LBM_F16NE = 3 };

enum {                      /* lbm_reduce: what                                  */
    LBM_RED_SUMS = 0,       /* sum_x Q_k(x)                        -> K doubles  */
    LBM_RED_RELL2 = 1,      /* ||Q_k - ref_k||_2 / ||ref_k||_2     -> K doubles  */
    LBM_RED_RELLINF = 2,    /* max|Q_k - ref_k| / max|ref_k|       -> K doubles  */
    LBM_RED_MAXSPEED = 3,   /* (dt/dx) max_x max_n |eig A_n(Q)|, and that value
                               divided by cs                      -> 2 doubles  */
    LBM_RED_NONFINITE = 4   /* number of non-finite populations    -> 1 double   */
};

/* Create a stepper (host only; no device work).
 *   system:  "swe2d"         shallow water (h, hu, hv), Sec. 3
 *            "advdiff_trk2d" scalar advection-diffusion(-reaction) with a
 *                            gradient tracker (c, G_c), Sec. 3
 *            "neohooke2d"    neo-Hookean elasticity (F00, F01, F10, F11, v0, v1), Sec. 3
 *            "nsf3d_trk17"   3D compressible NSF with 9 velocity-gradient and
 *                            3 temperature-gradient trackers (Sec. 3, the
 *                            homogenized NSF case at porosity 1, full tracker basis)
 *            "burgers2d"     inviscid Burgers (u), Sec. 3
 *            "euler2d"       compressible Euler (rho, rho u0, rho u1, E), ideal gas, Sec. 3
 *            "maxwell2d"     Maxwell, transverse-magnetic mode (E_z, H_x, H_y), Sec. 3
 *            "allencahn_trk2d" Allen-Cahn phase field with a gradient
 *                            tracker (phi, G_phi), Sec. 3
 *            "relhydro2d"    ideal ultrarelativistic fluid (E, S0, S1), c = 1, Sec. 3
 *            "nse_trk2d"     weakly compressible Navier-Stokes (rho, rho u0,
 *                            rho u1) with momentum-gradient trackers, Sec. 3
 *            "cnsf_trk2d"    2D compressible Navier-Stokes-Fourier (rho,
 *                            rho u0, rho u1, E) with conserved-field gradient
 *                            trackers (12 fields), Sec. 3
 *            "mhd_trk2d"     2D resistive MHD (rho, rho u0, rho u1, E, B0, B1;
 *                            B in Alfven units) with conserved-field gradient
 *                            trackers and the Powell source (18 fields), Sec. 3
 *            "hcnsf3d_trk14" 3D homogenized compressible NSF (rho, rho u, E,
 *                            sym grad u as 00, 11, 22, 01, 02, 12, grad T;
 *                            14 fields) with a prescribed per-cell porosity
 *                            and solid velocity ("coef" field), Sec. 3
 *            "gen_euler2d", "gen_advdiff_trk2d", "gen_cnsf_trk2d"
 *                            the same physics compiled from declared
 *                            conservation laws (Alg. 1: Split, Cascade,
 *                            Assemble; the functors are generated at build
 *                            time); parameters by their declared names
 *                            (gen_cnsf_trk2d: gamma, mu, kappa, R_gas, g_tau),
 *                            reference default the paper's MMS background; the
 *                            max-wave-speed reduction returns 0 for them
 *   Tracker layout (2D): tracker fields follow the conserved fields, two
 *   per tracked field in field order (G_q,0, G_q,1).
 *   lattice: "D2Q5" | "D2Q9" (2D systems) | "D3Q7" (3D systems)
 *   nx, ny, nz: grid; nz must be 1 in 2D (rows whose length is a multiple
 *   of 64 map onto whole wavefronts; any size is accepted).
 *   tau: relaxation time tau_LB of the conserved fields (> 1/2); dt, dx:
 *   time step and grid spacing (the flux enters the equilibrium times dt/dx).
 * Returns NULL on error (message via lbm_last_error(NULL)). */
lbm_state *lbm_create(const char *system, const char *lattice, int nx, int ny, int nz,
                      double tau, double dt, double dx);

/* Message of the last failed call on this handle, or of the last failed
 * lbm_create on this thread when h is NULL.  Never NULL. */
const char *lbm_last_error(const lbm_state *h);

/* Number of fields K and of lattice velocities Q. */
int lbm_num_fields(const lbm_state *h);
int lbm_num_velocities(const lbm_state *h);

/* Set a named scalar parameter before lbm_bind.
 *   swe2d:          g
 *   advdiff_trk2d:  ax, ay (advection velocity), nu (diffusivity D), R (reaction), g_tau
 *   neohooke2d:     rho0, mu_s, lambda_s
 *   nsf3d_trk17:    gamma, mu, kappa, g_tau, mms (0/1: built-in manufactured-
 *                   solution forcing), mms_amp, mms_rho0, mms_p0, mms_u0
 *   burgers2d:      (none)
 *   euler2d:        gamma (adiabatic index, default 1.4)
 *   maxwell2d:      c (wave speed, default 1)
 *   allencahn_trk2d: nu (interface diffusivity gamma), R (reaction rate r), g_tau
 *   relhydro2d:     (none)
 *   nse_trk2d:      cs_phys (physical sound speed), mu (dynamic viscosity), g_tau
 *   cnsf_trk2d:     gamma, mu (dynamic viscosity), kappa (heat conductivity K),
 *                   R_gas (T = p / (rho R_gas)), g_tau
 *   mhd_trk2d:      gamma, mu (dynamic viscosity), kappa (heat-flux coefficient
 *                   K, with T = p / rho), eta (magnetic diffusivity), g_tau
 *   hcnsf3d_trk14:  gamma, mu, kappa (T = p / rho), eta (drag time, > 0), g_tau
 *   all:            t0 (initial time); trt_lambda (>= 0; 0 = BGK, the default):
 *                   two-relaxation-time collision with this magic parameter
 *                   Lambda = (1/omega+ - 1/2)(1/omega- - 1/2): the parts of
 *                   each field's populations antisymmetric under c -> -c
 *                   (which carry the flux) relax at the field's BGK rate
 *                   omega-, the symmetric parts at omega+ (Sec. 2.3 names
 *                   such operators as consuming the same equilibria).  Not
 *                   with LBM_F16NE storage, the moment history or the
 *                   adjoint (LBM_EINVAL).
 *                   regularized (0 or 1; default 0): regularized collision
 *                   (Sec. 2.3, the Latt-Chopard operator with first-order
 *                   Hermite projection): each field's non-equilibrium part
 *                   is replaced by w_i c_i . Pi1 / cs^2, Pi1 its first
 *                   moment, before relaxing at the field's BGK rate, so
 *                   post_i = feq_i + (1 - omega) w_i c_i . Pi1 / cs^2.  The
 *                   first-order projection keeps the flux relaxation and
 *                   drops the symmetric non-equilibrium, which makes it
 *                   unstable near omega -> 2 on some flows.  Excludes
 *                   trt_lambda > 0, LBM_F16NE, the moment history and the
 *                   adjoint (LBM_EINVAL).
 *                   check_every (a step count N >= 0, default 0; may be
 *                   changed at any time): failure detection.  Outside the
 *                   sub-characteristic bound (Sec. 2.4.2) the scheme blows
 *                   up; with N > 0, lbm_step and lbm_step_record scan the
 *                   populations for non-finite values after every step whose
 *                   count is a multiple of N (one LBM_RED_NONFINITE
 *                   reduction, which synchronises the stream) and return
 *                   LBM_ENONFINITE at the first one that finds any; the step
 *                   counter then stands at that step.
 *                   check_subchar (0 or 1, default 1): the sub-characteristic
 *                   check of lbm_init_moments. */
int lbm_set_param(lbm_state *h, const char *name, double v);

/* Read a parameter in use: "dt", "dx", "lambda" (dt/dx), "tau", "omega"
 * (conserved fields), "omega_tracker", "tau_grad", "g_tau", "g", "t0",
 * "trt_lambda", "regularized", "check_every", and once bound "omega_plus" /
 * "omega_plus_tracker" (the
 * symmetric TRT rates; equal to omega / omega_tracker under BGK).  Under TRT
 * the kernels use a = (omega+ + omega-)/2 and b = (omega+ - omega-)/2, in
 * single precision with 2 - a on the 2^-24 grid and b rounded once; omega
 * and omega_plus then report a - b and a + b.
 * After lbm_bind with F32/F16 storage these are the values the kernels run
 * with: dt/dx is rounded once to float and 2 - omega to a multiple of 2^-24
 * (so that omega - 1 is exact in float), and dt, tau and the collision
 * rates are the values those roundings define.  LBM_EINVAL for an
 * unknown name. */
int lbm_get_param(const lbm_state *h, const char *name, double *v);

/* Population storage LBM_F64 / LBM_F32 / LBM_F16 / LBM_F16NE, before
 * lbm_bind.  Default: LBM_F32.  LBM_F16NE has no adjoint and no moment
 * history. */
int lbm_set_storage(lbm_state *h, int storage);

/* Reference state Q0 (K host doubles) of the shifted form, before lbm_bind.
 * For F32/F16 storage it is rounded to the nearest float; lbm_get_reference
 * returns the value in use.  Defaults: swe2d (1,0,0); advdiff (1,0,0);
 * neohooke2d (1,0,0,1,0,0); nsf3d_trk17 (1, u0,u0,u0, E0, 0...) from the
 * mms_* parameters; euler2d (1, 3, 3, 1/(gamma (gamma-1)) + 9), the
 * Mach-3 background of the paper's manufactured solution in units
 * rho0 = cs = 1; cnsf_trk2d (1, 3, 2, 1/(gamma (gamma-1)) + 13/2, 0...);
 * mhd_trk2d (1, 3, 3, 1/(gamma (gamma-1)) + 37/4, 1/2, 1/2, 0...);
 * hcnsf3d_trk14 (1, U0, U0, U0, 1/(gamma-1) + 3/2 U0^2, 0...) with
 * U0 = sqrt(gamma)/2 (Mach 1/2 per axis, p0 = rho0 = 1; its tracker
 * entries must be zero: LBM_EINVAL otherwise);
 * relhydro2d (3, 1.2, 1.2); nse_trk2d (1, 0...); burgers2d, maxwell2d,
 * allencahn_trk2d all zeros. */
int lbm_set_reference(lbm_state *h, const double *Q0);
int lbm_get_reference(const lbm_state *h, double *Q0_out);

/* Bytes the caller must provide: which = 0 one population buffer
 * (K*Q*nz*ceil(nx ny / 64)*64*sizeof(storage), the tile-blocked layout; for
 * LBM_F16NE the binary16 deviations in the same tile-blocked layout,
 * padded to 256 bytes, followed by K*cells floats of moments); which = 1
 * scratch for reductions. */
size_t lbm_required_bytes(const lbm_state *h, int which);

/* Bind caller-owned device memory: two population buffers (A/B, each
 * lbm_required_bytes(h,0) bytes, 256-byte aligned), the scratch buffer
 * (lbm_required_bytes(h,1)) and the hipStream_t all calls are ordered on
 * (NULL = default stream).  The library never frees them. */
int lbm_bind(lbm_state *h, void *pop_a, void *pop_b, void *aux, void *hip_stream);

/* Attach a per-cell device field (caller-owned, [NB][cells] in the
 * arithmetic type: double for F64 storage, float otherwise; NULL detaches):
 *   "grad_zb" (swe2d, NB = 2): topography gradient b = grad z_b, read by the
 *            source;
 *   "coef"   (hcnsf3d_trk14, NB = 4): porosity alpha in [0, 1] and solid
 *            velocity u_s, read by the flux and the source of every step
 *            and by lbm_init_moments (attach it before initialising; without
 *            it every cell is fluid, alpha = 1).  Not with LBM_F16NE.
 *   "source" (every system, NB = K): an explicit per-cell source added to
 *            S_k of every step (eq. lbe_update: evaluated by the caller at
 *            t + dt/2, e.g. a manufactured-solution forcing).  Not with
 *            LBM_F16NE.
 * The caller may rewrite a field between steps (on the bound stream) to
 * prescribe it in time. */
int lbm_set_field(lbm_state *h, const char *name, const void *dev_ptr);

/* Initialise the populations at the shifted equilibrium of the given fields
 * Q_dev ([K][cells] device doubles), computed in double and rounded once to
 * the storage type (supplement: populations start at the equilibrium of the
 * initial fields).  For F16 storage, chooses each field's power-of-two scale
 * from the initial populations.  Resets the step counter and time to t0.
 * Returns LBM_ESUBCHAR if (dt/dx) max |eig A_n| exceeds cs (Sec. 2.4.2). */
int lbm_init_moments(lbm_state *h, const double *Q_dev);

/* Advance n collide-and-stream steps (eq. lbe_update), one fused kernel per
 * step with pull streaming between the A/B buffers.  Asynchronous, unless
 * check_every is set (see lbm_set_param): then LBM_ENONFINITE reports
 * non-finite populations. */
int lbm_step(lbm_state *h, int n);

/* Like lbm_step, additionally writing the pre-collision moment deviations
 * dQ^m = Q^m - Q0 of each of the n steps to Q_hist_dev ([n][K][cells]
 * floats, or doubles for F64 storage): the recomputation pass of the
 * checkpointed adjoint. */
int lbm_step_record(lbm_state *h, int n, void *Q_hist_dev);

/* Moments Q_k(x) at the current time (eq. moments): absolute (Q0 + sum f*)
 * when absolute != 0, else the deviation; out_dtype LBM_F64 or LBM_F32;
 * Q_out_dev is [K][cells].  Asynchronous. */
int lbm_moments(lbm_state *h, void *Q_out_dev, int absolute, int out_dtype);

/* FP64 reductions over the grid (validation-section norms, Sec. 2.4.2
 * wave-speed bound), written to host_out; ref_dev ([K][cells] doubles) is
 * required for RELL2 / RELLINF.  Synchronises the bound stream. */
int lbm_reduce(lbm_state *h, int what, const double *ref_dev, double *host_out);

/* lbm_reduce without the bound workspace, for callers that cannot allocate
 * device memory (and so cannot size an aux buffer of their own): the same
 * reductions, same kernels and same results, with the partial sums kept in
 * a static device array of 295,488 bytes per GPU (2 x 18 x 1024 + 72
 * doubles: the largest system's partials and final slots).  The array is
 * part of the loaded library and lives until the process ends; its address
 * is looked up once per device, with that device current, on the first
 * call.  Arguments, results and errors as for lbm_reduce; LBM_EINVAL if the
 * reduction needed more than the static array (no system does).  Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (from
 * several threads or handles at once) race and must be serialised by the
 * caller.  Allocates nothing; synchronises the bound stream. */
int lbm_reduce_static(lbm_state *h, int what, const double *ref_dev, double *host_out);

/* Current step count and time. */
long long lbm_step_count(const lbm_state *h);
double lbm_time(const lbm_state *h);

/* Discrete adjoint of the step (not in the paper; derived from eq.
 * lbe_update).  Adjoint populations lam[K][Q][cells] hold dL/df*_{k,i}(x)
 * of the pre-collision populations, in the arithmetic type.
 *
 * lbm_adjoint_seed: lam_{k,i}(x) = dLdQ_k(x) for every i, from the loss
 * gradient w.r.t. the moments at the final time, dLdQ_dev [K][cells].
 *
 * lbm_adjoint_step: n steps backwards, lam^m = J_m^T lam^{m+1}, using the
 * recorded moment deviations of lbm_step_record (Q_hist_dev, [n][K][cells],
 * entry j = step m0 + j) from last to first.  lam^{m0+n} enters in lam_a;
 * buffers alternate, so lam^{m0} leaves in lam_a when n is even and in
 * lam_b when n is odd.  grad_field_dev, if non-NULL, accumulates the
 * gradient w.r.t. the attached source field (swe2d: dL/d grad_zb,
 * [2][cells]).
 *
 * lbm_adjoint_to_initial: dL/dQ^0 [K][cells] (doubles) from lam^0 through the
 * equilibrium initialisation at the initial fields Q_init_dev (doubles). */
int lbm_adjoint_seed(lbm_state *h, const void *dLdQ_dev, void *lam_dev);
int lbm_adjoint_step(lbm_state *h, int n, void *lam_a, void *lam_b, const void *Q_hist_dev,
                     void *grad_field_dev);
int lbm_adjoint_to_initial(lbm_state *h, const void *lam0_dev, const double *Q_init_dev,
                           double *dLdQ0_dev);

/* Checkpoint: serialise the current populations and the handle's state
 * (system, lattice, grid, storage, step, time, parameters, Q0, F16 scales)
 * into host_buf.  lbm_save with host_buf == NULL returns the size needed in
 * *n_inout; lbm_load restores a buffer written by lbm_save into a handle of
 * the same system, lattice, grid and storage.  Both synchronise. */
int lbm_save(lbm_state *h, void *host_buf, size_t *n_inout);
int lbm_load(lbm_state *h, const void *host_buf, size_t n);

/* Device-side checkpoints for the checkpointed adjoint: lbm_snapshot copies
 * the current populations (lbm_required_bytes(h,0) bytes) to dev_buf;
 * lbm_restore copies them back and sets the step counter to `step`.
 * Asynchronous on the bound stream. */
int lbm_snapshot(lbm_state *h, void *dev_buf);
int lbm_restore(lbm_state *h, const void *dev_buf, long long step);

/* Bandwidth probes (measurement only; no part of a step).
 *
 * lbm_bw_copy copies n bytes src -> dst, 16 bytes per lane with
 * non-temporal loads and stores: the best plain-copy rate of the part.
 *
 * lbm_bw_streams reproduces the memory-access pattern of the 2D D2Q9 step
 * without its arithmetic: src and dst each hold 9 * fields float planes of
 * nx * ny cells in the tile-blocked population layout ([tiles][9 fields][64],
 * byte size 36 fields ceil(nx ny / 64) 64); every cell (x, y) reads plane j
 * at the periodic pull position (x, y) - c_(j mod 9) (D2Q9 order of the
 * population layout) and writes it to plane j at (x, y), one 4-byte element
 * per lane and plane, all loads of a cell issued before its stores.  Like
 * the step, when the two buffers exceed the 256 MiB last-level cache it
 * stores non-temporally and (at most 300 bytes per cell, fields 3) runs its
 * tiles in dispatch order, else in XCD-contiguous runs.  fields must be 3
 * or 6; LBM_EINVAL otherwise or for null pointers or nx, ny < 1.
 * Asynchronous on hip_stream.  With the step's own sizes it measures what
 * the memory system delivers for that access pattern. */
int lbm_bw_copy(void *dst, const void *src, size_t n, void *hip_stream);
int lbm_bw_streams(void *dst, const void *src, int nx, int ny, int fields, void *hip_stream);

/* lbm_bw_streams3 is the same probe for the 3D D3Q7 step: src and dst each
 * hold 7 * fields float planes of nx * ny * nz cells in the step's
 * tile-blocked layout ([nz][tiles][7 fields][64], each z-slab padded to
 * whole tiles: byte size 28 fields ceil(nx ny / 64) 64 nz); cell (x, y, z)
 * reads plane j at the periodic pull position (x, y, z) - c_(j mod 7) (D3Q7
 * order of the population layout) and writes it, non-temporally, to plane
 * j at (x, y, z).  It is launched in the 17-field step's shape: 512-thread
 * workgroups, one per CU.  fields must be 14 or 17; LBM_EINVAL otherwise,
 * for null pointers, nx, ny, nz < 1 or a slab beyond 4 GiB.  Asynchronous
 * on hip_stream. */
int lbm_bw_streams3(void *dst, const void *src, int nx, int ny, int nz, int fields, void *hip_stream);

/* Release the handle (does not touch bound buffers). */
void lbm_destroy(lbm_state *h);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
