// Internal declarations shared by the kernels (kernels.hip) and the C ABI
// (lbm_api.cpp).  Not installed; the public interface is include/lbm.h.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "systems.hpp"

enum {
    SYS_ADVDIFF = 0, SYS_SWE = 1, SYS_NEOHOOKE = 2, SYS_NSF17 = 3, SYS_BURGERS = 4, SYS_EULER = 5,
    SYS_MAXWELL = 6, SYS_ALLENCAHN = 7, SYS_RELHYDRO = 8, SYS_NSE = 9, SYS_CNSF2D = 10,
    SYS_MHD = 11,
    SYS_HCNSF = 12,
    SYS_GEN0 = 100             // generated systems: SYS_GEN0 + index in the registry
};
enum { LAT_D2Q5 = 0, LAT_D2Q9 = 1, LAT_D3Q7 = 2 };

#ifndef LBM_BLOCK
#define LBM_BLOCK 256
#endif
#ifndef LBM_XCD_REMAP
#define LBM_XCD_REMAP 1                 // consecutive tiles on one XCD
#endif
constexpr int kBlock = LBM_BLOCK;    // threads per workgroup (wave64 multiples)
// Population buffers larger than this together (A + B) are written with
// non-temporal stores: MI355X's Infinity Cache holds 256 MiB.
constexpr size_t kLastLevelCacheBytes = (size_t)256 << 20;
constexpr int kRedBlocks = 1024;     // workgroups of the first reduction pass
// Population layout: each z-slab's nx*ny cells are cut into tiles of kTile
// consecutive cells (x fastest, rows continue into the next tile), and a
// tile keeps all K*Q populations of its cells together,
// [z][tile][K][Q][kTile]: one wavefront's 64 cells of one population are one
// contiguous 256-byte (FP32) run, and all of a wavefront's populations one
// contiguous block.  The last tile of a slab is padded.
constexpr int kTile = 64;
__host__ __device__ inline long long padded_plane(long long P) { return (P + kTile - 1) / kTile * kTile; }

// Manufactured-solution forcing of the 3D NSF system (conserved rows).
template <class R>
struct MmsParams {
    int on;
    R amp, rho0, p0, u0, cbar2;      // shape parameters of the exact fields
    R t;                              // evaluation time t_n + dt/2
    R k;                              // wavenumber 2 pi (phases evaluated as sinpi(2 X))
    R dx;
};

// Everything one kernel launch needs, by value (kernel arguments).
template <class R>
struct KParams {
    int nx, ny, nz;
    long long C;                      // cells
    R lam_cs2;                        // (dt/dx) / cs^2
    R lam;                            // dt/dx
    R dt;
    R omega[LBM_MAXK];                // collision rate per field
    R delta[LBM_MAXK];                // 2 - omega
    R c1[LBM_MAXK];                   // 1 - delta = omega - 1 (exactly representable)
    R c2[LBM_MAXK];                   // 2 - delta = omega
    R tb[LBM_MAXK];                   // two-relaxation-time: (omega+ - omega-) / 2 (c1 = a - 1, c2 = a,
                                      // a = (omega+ + omega-) / 2); zero under BGK
    float scale[LBM_MAXK];            // storage = value * scale (F16 only)
    float inv_scale[LBM_MAXK];
    Phys<R> phys;
    const R *b;                       // per-cell source field [D][C] or null
    const R *sext;                    // per-cell explicit source [K][C] added to S_k, or null
    MmsParams<R> mms;
};

struct lbm_state_impl;

// Launchers of one (system, lattice, storage) instantiation.
struct Launchers {
    int K, Q, D;
    size_t store_bytes;               // bytes per stored population
    hipError_t (*step)(const lbm_state_impl &, const void *fin, void *fout, void *qhist, hipStream_t);
    hipError_t (*init)(const lbm_state_impl &, const double *Q, void *fout, hipStream_t);
    hipError_t (*init_absmax)(const lbm_state_impl &, const double *Q, double *partial, hipStream_t);
    hipError_t (*moments)(const lbm_state_impl &, const void *fin, void *out, int absolute, int out_dtype,
                          hipStream_t);
    hipError_t (*reduce)(const lbm_state_impl &, const void *fin, int what, const double *ref, double *aux,
                         hipStream_t);
    hipError_t (*adj_seed)(const lbm_state_impl &, const void *dLdQ, void *lam, hipStream_t);
    hipError_t (*adj_step)(const lbm_state_impl &, const void *lam_in, void *lam_out, const void *qhist,
                           void *grad_b, hipStream_t);
    hipError_t (*adj_init)(const lbm_state_impl &, const void *lam0, const double *Q, double *dQ0,
                           hipStream_t);
};

const Launchers *lbm_launchers(int sys, int lat, int storage);
// per system family (sys_*.hip); nullptr for an unsupported lattice
const Launchers *lbm_launchers_swe(int lat, int storage);
const Launchers *lbm_launchers_advdiff(int lat, int storage);
const Launchers *lbm_launchers_neohooke(int lat, int storage);
const Launchers *lbm_launchers_nsf17(int lat, int storage);
const Launchers *lbm_launchers_burgers(int lat, int storage);
const Launchers *lbm_launchers_euler(int lat, int storage);
const Launchers *lbm_launchers_maxwell(int lat, int storage);
const Launchers *lbm_launchers_allencahn(int lat, int storage);
const Launchers *lbm_launchers_relhydro(int lat, int storage);
const Launchers *lbm_launchers_nse(int lat, int storage);
const Launchers *lbm_launchers_cnsf2d(int lat, int storage);
const Launchers *lbm_launchers_mhd(int lat, int storage);
const Launchers *lbm_launchers_hcnsf(int lat, int storage);
// generated systems (sys_gen.hip): launchers and registry entries
const Launchers *lbm_launchers_gen(int gen, int lat, int storage);
int lbm_gen_count();
const char *lbm_gen_name(int gen);
int lbm_gen_fields(int gen, int *D, int *n_conserved, int *npar);
const char *lbm_gen_param_name(int gen, int j);
double lbm_gen_param_default(int gen, int j);
double lbm_gen_reference(int gen, int k);
const Launchers *lbm_launchers_ne(int sys, int lat);   // storage LBM_F16NE
hipError_t lbm_launch_copy(void *dst, const void *src, size_t n, hipStream_t s);
hipError_t lbm_launch_streams(void *dst, const void *src, int nx, int ny, int fields, hipStream_t s);
hipError_t lbm_launch_streams3(void *dst, const void *src, int nx, int ny, int nz, int fields, hipStream_t s);

// Host-side state behind the opaque lbm_state handle.
struct lbm_state_impl {
    int sys = 0, lat = 0, storage = 1;
    int nx = 0, ny = 0, nz = 1;
    long long C = 0;
    int K = 0, Q = 0, D = 0;
    double tau = 0, dt = 0, dx = 0, cs2 = 0;
    double omega_c = 0, omega_t = 0;     // collision rates in use (conserved, trackers)
    // physical parameters (host, double)
    double g = 1.0, ax = 0, ay = 0, nu = 0, react = 0, g_tau = -1;
    double gamma = 1.4, mu = 0, kappa = 0;
    double rho0_el = 1.0, mu_s = 1.0, lam_s = 1.0;
    double c_light = 1.0;
    double cs_phys = 1.0;
    double R_gas = 1.0;
    double eta_drag = 0.1;                 // homogenized NSF: drag time eta
    double trt_lambda = 0.0;               // two-relaxation-time magic parameter (0: BGK)
    bool regularized = false;              // regularized collision (first-order Hermite projection)
    double gen_par[16] = {};               // generated systems: declared parameters
    double trt_a[2] = {0, 0}, trt_b[2] = {0, 0};   // TRT (a, b) of conserved fields, trackers
    int mms_on = 0;
    double mms_amp = 0.05, mms_rho0 = 1.0, mms_p0 = 1.0, mms_u0 = 0.0;
    double t0 = 0.0;
    int check_subchar = 1;
    long long check_every = 0;             // non-finite scan every N steps (0: never)
    int use_graphs = 1;                    // replay runs of small-grid launches from HIP graphs
    long long epoch = 0;                   // advanced whenever kernel arguments may change
    void *graphs = nullptr;                // captured launch graphs (lbm_api.cpp)
    double Q0[LBM_MAXK] = {0};
    bool q0_set = false;
    int scale_exp[LBM_MAXK] = {0};
    // device binding
    void *pop[2] = {nullptr, nullptr};
    int cur = 0;
    void *aux = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
    const void *field_b = nullptr;
    const void *field_src = nullptr;         // explicit per-cell source [K][cells]
    // time
    long long nsteps = 0;
    const Launchers *L = nullptr;
    std::string err;

    template <class R> KParams<R> kparams(double t_half) const;
};
