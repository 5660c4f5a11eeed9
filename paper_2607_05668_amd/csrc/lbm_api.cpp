// C ABI of the collide-and-stream library (declared in include/lbm.h):
// handle management, parameter derivation and launch ordering.  All
// numerical work is done by the kernels in kernels.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "impl.hpp"
#include "lbm.h"

struct lbm_state : lbm_state_impl {};

namespace {

thread_local std::string g_create_error = "no error";

int fail(lbm_state *h, int code, const std::string &msg)
{
    if (h) h->err = msg;
    return code;
}

int hipfail(lbm_state *h, hipError_t e, const char *where)
{
    return fail(h, LBM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

int system_id(const char *s)
{
    if (!s) return -1;
    if (!std::strcmp(s, "advdiff_trk2d")) return SYS_ADVDIFF;
    if (!std::strcmp(s, "swe2d")) return SYS_SWE;
    if (!std::strcmp(s, "neohooke2d")) return SYS_NEOHOOKE;
    if (!std::strcmp(s, "nsf3d_trk17")) return SYS_NSF17;
    if (!std::strcmp(s, "burgers2d")) return SYS_BURGERS;
    if (!std::strcmp(s, "euler2d")) return SYS_EULER;
    if (!std::strcmp(s, "maxwell2d")) return SYS_MAXWELL;
    if (!std::strcmp(s, "allencahn_trk2d")) return SYS_ALLENCAHN;
    if (!std::strcmp(s, "relhydro2d")) return SYS_RELHYDRO;
    if (!std::strcmp(s, "nse_trk2d")) return SYS_NSE;
    if (!std::strcmp(s, "cnsf_trk2d")) return SYS_CNSF2D;
    if (!std::strcmp(s, "mhd_trk2d")) return SYS_MHD;
    if (!std::strcmp(s, "hcnsf3d_trk14")) return SYS_HCNSF;
    for (int g = 0; g < lbm_gen_count(); ++g)
        if (!std::strcmp(s, lbm_gen_name(g))) return SYS_GEN0 + g;
    return -1;
}

int lattice_id(const char *s)
{
    if (!s) return -1;
    if (!std::strcmp(s, "D2Q5")) return LAT_D2Q5;
    if (!std::strcmp(s, "D2Q9")) return LAT_D2Q9;
    if (!std::strcmp(s, "D3Q7")) return LAT_D3Q7;
    return -1;
}

const int kSysK[13] = {3, 3, 6, 17, 1, 4, 3, 3, 3, 7, 12, 18, 14};
const int kSysD[13] = {2, 2, 2, 3, 2, 2, 2, 2, 2, 2, 2, 2, 3};

// fields, dimension and conserved-field count of any system id
int sys_K(int sys)
{
    if (sys < SYS_GEN0) return kSysK[sys];
    int d, nc, np;
    return lbm_gen_fields(sys - SYS_GEN0, &d, &nc, &np);
}
int sys_D(int sys)
{
    if (sys < SYS_GEN0) return kSysD[sys];
    int d, nc, np;
    lbm_gen_fields(sys - SYS_GEN0, &d, &nc, &np);
    return d;
}
int gen_conserved(int sys)
{
    int d, nc, np;
    lbm_gen_fields(sys - SYS_GEN0, &d, &nc, &np);
    return nc;
}
const int kLatQ[3] = {5, 9, 7};
const int kLatD[3] = {2, 2, 3};
const double kLatCs2[3] = {1.0 / 3.0, 1.0 / 3.0, 1.0 / 4.0};

// Reference state of the 3D NSF system from its manufactured-solution
// background: rho0, rho0 u0 (per axis), E0 = p0/(gamma-1) + 3/2 rho0 u0^2.
void nsf_default_reference(lbm_state *h)
{
    std::memset(h->Q0, 0, sizeof h->Q0);
    h->Q0[0] = h->mms_rho0;
    for (int a = 0; a < 3; ++a) h->Q0[1 + a] = h->mms_rho0 * h->mms_u0;
    h->Q0[4] = h->mms_p0 / (h->gamma - 1.0) + 1.5 * h->mms_rho0 * h->mms_u0 * h->mms_u0;
}

// Reference state of the Euler system: the background of the paper's
// manufactured solution in units rho0 = cs = 1 (Mach 3 per axis):
// rho0 = 1, m0 = (3, 3), E0 = p0 / (gamma - 1) + 9 with p0 = 1 / gamma.
void euler_default_reference(lbm_state *h)
{
    std::memset(h->Q0, 0, sizeof h->Q0);
    h->Q0[0] = 1.0;
    h->Q0[1] = 3.0;
    h->Q0[2] = 3.0;
    h->Q0[3] = (1.0 / h->gamma) / (h->gamma - 1.0) + 9.0;
}

// Reference state of the 2D compressible NSF system: the background of the
// paper's manufactured solution in units rho0 = cs = 1 (Mach 3 and 2 per
// axis): rho0 = 1, m0 = (3, 2), E0 = p0 / (gamma - 1) + 13/2, p0 = 1/gamma,
// trackers zero.
void cnsf2d_default_reference(lbm_state *h)
{
    std::memset(h->Q0, 0, sizeof h->Q0);
    h->Q0[0] = 1.0;
    h->Q0[1] = 3.0;
    h->Q0[2] = 2.0;
    h->Q0[3] = (1.0 / h->gamma) / (h->gamma - 1.0) + 6.5;
}

// Reference state of the 2D resistive MHD system: the background of the
// paper's manufactured solution in units rho0 = cs = 1 (Mach 3 per axis,
// field (1/2, 1/2) in Alfven units): E0 = p0 / (gamma - 1) + 9 + 1/4.
void mhd_default_reference(lbm_state *h)
{
    std::memset(h->Q0, 0, sizeof h->Q0);
    h->Q0[0] = 1.0;
    h->Q0[1] = 3.0;
    h->Q0[2] = 3.0;
    h->Q0[3] = (1.0 / h->gamma) / (h->gamma - 1.0) + 9.25;
    h->Q0[4] = 0.5;
    h->Q0[5] = 0.5;
}

// Reference state of the 3D homogenized NSF system: the background of the
// paper's manufactured solution in units rho0 = cs = 1 (isothermal cs,
// p0 = 1): drift Ma sqrt(gamma) per axis with Ma = 1/2,
// E0 = p0 / (gamma - 1) + 3/2 rho0 U0^2, trackers zero.
void hcnsf_default_reference(lbm_state *h)
{
    std::memset(h->Q0, 0, sizeof h->Q0);
    const double u0 = 0.5 * std::sqrt(h->gamma);
    h->Q0[0] = 1.0;
    for (int a = 0; a < 3; ++a) h->Q0[1 + a] = u0;
    h->Q0[4] = 1.0 / (h->gamma - 1.0) + 1.5 * u0 * u0;
}

void default_reference(lbm_state *h)
{
    std::memset(h->Q0, 0, sizeof h->Q0);
    switch (h->sys) {
    case SYS_SWE: h->Q0[0] = 1.0; break;
    case SYS_ADVDIFF: h->Q0[0] = 1.0; break;
    case SYS_NEOHOOKE: h->Q0[0] = 1.0; h->Q0[3] = 1.0; break;
    case SYS_NSF17: nsf_default_reference(h); break;
    case SYS_BURGERS: break;                       // u0 = 0
    case SYS_RELHYDRO: h->Q0[0] = 3.0; h->Q0[1] = 1.2; h->Q0[2] = 1.2; break;
    case SYS_NSE: h->Q0[0] = 1.0; break;
    case SYS_CNSF2D: cnsf2d_default_reference(h); break;
    case SYS_MHD: mhd_default_reference(h); break;
    case SYS_HCNSF: hcnsf_default_reference(h); break;
    case SYS_EULER: euler_default_reference(h); break;
    default:
        if (h->sys >= SYS_GEN0)
            for (int k = 0; k < h->K; ++k) h->Q0[k] = lbm_gen_reference(h->sys - SYS_GEN0, k);
        break;
    }
}

bool has_trackers(int sys)
{
    return sys == SYS_ADVDIFF || sys == SYS_NSF17 || sys == SYS_ALLENCAHN || sys == SYS_NSE || sys == SYS_CNSF2D ||
           sys == SYS_MHD || sys == SYS_HCNSF || (sys >= SYS_GEN0 && gen_conserved(sys) < sys_K(sys));
}

size_t arith_bytes(const lbm_state *h) { return h->storage == LBM_F64 ? 8 : 4; }

size_t aux_bytes() { return sizeof(double) * ((size_t)2 * LBM_MAXK * kRedBlocks + 4 * LBM_MAXK); }

int check_ready(lbm_state *h)
{
    if (!h) return LBM_EINVAL;
    if (!h->bound) return fail(h, LBM_ENOTBOUND, "lbm_bind has not been called");
    return LBM_OK;
}

struct SaveHeader {
    char magic[8];
    int32_t version, sys, lat, storage, nx, ny, nz, K, Q;
    int64_t nsteps;
    double t0, tau, dt, dx;
    double Q0[LBM_MAXK];
    int32_t scale_exp[LBM_MAXK];
    uint64_t payload;
};

// ------------------------------------------------ launch batching ----
// On small grids a step kernel lasts a few microseconds, about as long as
// its launch from the host.  There the launches of a run of steps are
// captured once into a HIP graph (kernel nodes only) and replayed with one
// call.  A captured launch keeps the arguments it was captured with, so a
// graph is keyed by everything they depend on: the buffers, the history
// slice, the A/B parity and a parameter epoch that set_param, set_field,
// init_moments and load advance.  Kernels whose arguments change from step
// to step (the in-kernel manufactured forcing reads the time) are never
// captured; with failure detection on, steps run one by one.
constexpr long long kGraphMaxCells = 1ll << 20;  // above this a launch is long against its overhead
constexpr int kGraphMinLaunches = 4;
constexpr int kGraphChunk = 64;                   // launches per graph
constexpr size_t kGraphCacheSize = 16;

struct GraphKey {
    int kind, len, cur;
    long long epoch;
    const void *p[4];
    bool operator==(const GraphKey &o) const
    {
        return kind == o.kind && len == o.len && cur == o.cur && epoch == o.epoch && p[0] == o.p[0] &&
               p[1] == o.p[1] && p[2] == o.p[2] && p[3] == o.p[3];
    }
};

struct GraphCache {
    hipStream_t capture = nullptr;                   // private stream, default priority, used only to capture
    std::vector<std::pair<GraphKey, hipGraphExec_t>> entries;   // oldest first
    ~GraphCache()
    {
        for (auto &e : entries) (void)hipGraphExecDestroy(e.second);
        if (capture) (void)hipStreamDestroy(capture);
    }
};

GraphCache &graphs(lbm_state *h)
{
    if (!h->graphs) h->graphs = new GraphCache();
    return *(GraphCache *)h->graphs;
}

bool batch_launches(const lbm_state *h, int n)
{
    return h->use_graphs && n >= kGraphMinLaunches && h->C <= kGraphMaxCells &&
           !(h->sys == SYS_NSF17 && h->mms_on) && h->check_every == 0;
}

// Replay the graph of `key`, capturing it first with enqueue(stream) if it
// is not cached.
template <class F>
int replay(lbm_state *h, const GraphKey &key, F &&enqueue)
{
    GraphCache &gc = graphs(h);
    hipGraphExec_t exec = nullptr;
    for (auto &e : gc.entries)
        if (e.first == key) exec = e.second;
    hipError_t e;
    if (!exec) {
        if (!gc.capture) {
            e = hipStreamCreateWithFlags(&gc.capture, hipStreamNonBlocking);
            if (e != hipSuccess) return hipfail(h, e, "graph stream");
        }
        e = hipStreamBeginCapture(gc.capture, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hipfail(h, e, "graph capture");
        const hipError_t le = enqueue(gc.capture);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(gc.capture, &graph);
        if (le != hipSuccess || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hipfail(h, le != hipSuccess ? le : e, "graph capture");
        }
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hipfail(h, e, "graph instantiate");
        if (gc.entries.size() >= kGraphCacheSize) {
            (void)hipGraphExecDestroy(gc.entries.front().second);
            gc.entries.erase(gc.entries.begin());
        }
        gc.entries.emplace_back(key, exec);
    }
    e = hipGraphLaunch(exec, h->stream);
    return e == hipSuccess ? LBM_OK : hipfail(h, e, "graph launch");
}

}  // namespace

extern "C" {

lbm_state *lbm_create(const char *system, const char *lattice, int nx, int ny, int nz, double tau, double dt,
                      double dx)
{
    const int sys = system_id(system), lat = lattice_id(lattice);
    if (sys < 0) {
        g_create_error = std::string("unknown system '") + (system ? system : "(null)") + "'";
        return nullptr;
    }
    if (lat < 0) {
        g_create_error = std::string("unknown lattice '") + (lattice ? lattice : "(null)") + "'";
        return nullptr;
    }
    if (sys_D(sys) != kLatD[lat]) {
        g_create_error = "lattice dimension does not match the system";
        return nullptr;
    }
    if (sys == SYS_NSF17 && lat != LAT_D3Q7) {
        g_create_error = "nsf3d_trk17 runs on D3Q7";
        return nullptr;
    }
    if (nx <= 0 || ny <= 0 || nz <= 0 || (sys_D(sys) == 2 && nz != 1)) {
        g_create_error = "invalid grid (nz must be 1 in 2D)";
        return nullptr;
    }
    const long long C = (long long)nx * ny * nz;
    if ((long long)sys_K(sys) * kLatQ[lat] * C >= (1LL << 40)) {
        g_create_error = "grid too large";
        return nullptr;
    }
    if (!(tau > 0.5) || !(dt > 0) || !(dx > 0) || !std::isfinite(tau) || !std::isfinite(dt) || !std::isfinite(dx)) {
        g_create_error = "need tau > 1/2, dt > 0, dx > 0";
        return nullptr;
    }
    lbm_state *h = new lbm_state();
    h->sys = sys;
    h->lat = lat;
    h->nx = nx;
    h->ny = ny;
    h->nz = nz;
    h->C = C;
    h->K = sys_K(sys);
    if (sys >= SYS_GEN0) {
        int d, nc, np;
        lbm_gen_fields(sys - SYS_GEN0, &d, &nc, &np);
        for (int j = 0; j < np; ++j) h->gen_par[j] = lbm_gen_param_default(sys - SYS_GEN0, j);
    }
    h->Q = kLatQ[lat];
    h->D = kLatD[lat];
    h->tau = tau;
    h->dt = dt;
    h->dx = dx;
    h->cs2 = kLatCs2[lat];
    h->storage = LBM_F32;
    default_reference(h);
    h->err = "no error";
    return h;
}

const char *lbm_last_error(const lbm_state *h) { return h ? h->err.c_str() : g_create_error.c_str(); }

int lbm_num_fields(const lbm_state *h) { return h ? h->K : 0; }
int lbm_num_velocities(const lbm_state *h) { return h ? h->Q : 0; }

int lbm_set_param(lbm_state *h, const char *name, double v)
{
    if (!h || !name) return LBM_EINVAL;
    if (!std::isfinite(v)) return fail(h, LBM_EINVAL, "parameter value is not finite");
    const std::string n(name);
    h->epoch += 1;                      // captured launches may hold the old value
    if (n == "graphs") {
        if (v != 0.0 && v != 1.0) return fail(h, LBM_EINVAL, "graphs is 0 or 1");
        h->use_graphs = v != 0.0;
        return LBM_OK;
    }
    if (n == "t0") { h->t0 = v; return LBM_OK; }
    if (n == "regularized") {
        if (h->bound) return fail(h, LBM_EINVAL, "parameters are fixed once bound");
        if (v != 0.0 && v != 1.0) return fail(h, LBM_EINVAL, "regularized is 0 or 1");
        h->regularized = v != 0.0;
        return LBM_OK;
    }
    if (n == "trt_lambda") {
        if (h->bound) return fail(h, LBM_EINVAL, "parameters are fixed once bound");
        if (!(v >= 0)) return fail(h, LBM_EINVAL, "trt_lambda must be >= 0 (0: BGK)");
        h->trt_lambda = v;
        return LBM_OK;
    }
    if (n == "check_subchar") { h->check_subchar = v != 0.0; return LBM_OK; }
    if (n == "check_every") {
        if (!(v >= 0) || v != std::floor(v) || v > 1e15) return fail(h, LBM_EINVAL, "check_every is a step count >= 0");
        h->check_every = (long long)v;
        return LBM_OK;
    }
    if (h->bound && n != "mms") return fail(h, LBM_EINVAL, "parameters are fixed once bound");
    if (h->sys >= SYS_GEN0) {
        const int g = h->sys - SYS_GEN0;
        int d, nc, np;
        lbm_gen_fields(g, &d, &nc, &np);
        for (int j = 0; j < np; ++j)
            if (n == lbm_gen_param_name(g, j)) { h->gen_par[j] = v; return LBM_OK; }
        if (nc < h->K && n == "g_tau") {
            if (!(v > 0)) return fail(h, LBM_EINVAL, "g_tau must be positive");
            h->g_tau = v;
            return LBM_OK;
        }
    }
    switch (h->sys) {
    case SYS_SWE:
        if (n == "g") { h->g = v; return LBM_OK; }
        break;
    case SYS_ADVDIFF:
        if (n == "ax") { h->ax = v; return LBM_OK; }
        if (n == "ay") { h->ay = v; return LBM_OK; }
        if (n == "nu") { h->nu = v; return LBM_OK; }
        if (n == "R") { h->react = v; return LBM_OK; }
        if (n == "g_tau") {
            if (!(v > 0)) return fail(h, LBM_EINVAL, "g_tau must be positive");
            h->g_tau = v;
            return LBM_OK;
        }
        break;
    case SYS_NEOHOOKE:
        if (n == "rho0") { if (!(v > 0)) return fail(h, LBM_EINVAL, "rho0 must be positive"); h->rho0_el = v; return LBM_OK; }
        if (n == "mu_s") { h->mu_s = v; return LBM_OK; }
        if (n == "lambda_s") { h->lam_s = v; return LBM_OK; }
        break;
    case SYS_BURGERS:
        break;
    case SYS_MAXWELL:
        if (n == "c") {
            if (!(v > 0)) return fail(h, LBM_EINVAL, "c must be positive");
            h->c_light = v;
            return LBM_OK;
        }
        break;
    case SYS_RELHYDRO:
        break;
    case SYS_HCNSF:
        if (n == "gamma") {
            if (!(v > 1)) return fail(h, LBM_EINVAL, "gamma must exceed 1");
            h->gamma = v;
            if (!h->q0_set) hcnsf_default_reference(h);
            return LBM_OK;
        }
        if (n == "mu") { h->mu = v; return LBM_OK; }
        if (n == "kappa") { h->kappa = v; return LBM_OK; }
        if (n == "eta") {
            if (!(v > 0)) return fail(h, LBM_EINVAL, "eta must be positive");
            h->eta_drag = v;
            return LBM_OK;
        }
        if (n == "g_tau") {
            if (!(v > 0)) return fail(h, LBM_EINVAL, "g_tau must be positive");
            h->g_tau = v;
            return LBM_OK;
        }
        break;
    case SYS_MHD:
        if (n == "gamma") {
            if (!(v > 1)) return fail(h, LBM_EINVAL, "gamma must exceed 1");
            h->gamma = v;
            if (!h->q0_set) mhd_default_reference(h);
            return LBM_OK;
        }
        if (n == "mu") { h->mu = v; return LBM_OK; }
        if (n == "kappa") { h->kappa = v; return LBM_OK; }
        if (n == "eta") { h->nu = v; return LBM_OK; }
        if (n == "g_tau") {
            if (!(v > 0)) return fail(h, LBM_EINVAL, "g_tau must be positive");
            h->g_tau = v;
            return LBM_OK;
        }
        break;
    case SYS_CNSF2D:
        if (n == "gamma") {
            if (!(v > 1)) return fail(h, LBM_EINVAL, "gamma must exceed 1");
            h->gamma = v;
            if (!h->q0_set) cnsf2d_default_reference(h);
            return LBM_OK;
        }
        if (n == "mu") { h->mu = v; return LBM_OK; }
        if (n == "kappa") { h->kappa = v; return LBM_OK; }
        if (n == "R_gas") {
            if (!(v > 0)) return fail(h, LBM_EINVAL, "R_gas must be positive");
            h->R_gas = v;
            return LBM_OK;
        }
        if (n == "g_tau") {
            if (!(v > 0)) return fail(h, LBM_EINVAL, "g_tau must be positive");
            h->g_tau = v;
            return LBM_OK;
        }
        break;
    case SYS_NSE:
        if (n == "cs_phys") {
            if (!(v > 0)) return fail(h, LBM_EINVAL, "cs_phys must be positive");
            h->cs_phys = v;
            return LBM_OK;
        }
        if (n == "mu") { h->mu = v; return LBM_OK; }
        if (n == "g_tau") {
            if (!(v > 0)) return fail(h, LBM_EINVAL, "g_tau must be positive");
            h->g_tau = v;
            return LBM_OK;
        }
        break;
    case SYS_ALLENCAHN:
        if (n == "nu") { h->nu = v; return LBM_OK; }
        if (n == "R") { h->react = v; return LBM_OK; }
        if (n == "g_tau") {
            if (!(v > 0)) return fail(h, LBM_EINVAL, "g_tau must be positive");
            h->g_tau = v;
            return LBM_OK;
        }
        break;
    case SYS_EULER:
        if (n == "gamma") {
            if (!(v > 1)) return fail(h, LBM_EINVAL, "gamma must exceed 1");
            h->gamma = v;
            if (!h->q0_set) euler_default_reference(h);
            return LBM_OK;
        }
        break;
    case SYS_NSF17:
        if (n == "gamma") { if (!(v > 1)) return fail(h, LBM_EINVAL, "gamma must exceed 1"); h->gamma = v; if (!h->q0_set) nsf_default_reference(h); return LBM_OK; }
        if (n == "mu") { h->mu = v; return LBM_OK; }
        if (n == "kappa") { h->kappa = v; return LBM_OK; }
        if (n == "g_tau") {
            if (!(v > 0)) return fail(h, LBM_EINVAL, "g_tau must be positive");
            h->g_tau = v;
            return LBM_OK;
        }
        if (n == "mms") { h->mms_on = v != 0.0; return LBM_OK; }
        if (n == "mms_amp") { h->mms_amp = v; return LBM_OK; }
        if (n == "mms_rho0") { h->mms_rho0 = v; if (!h->q0_set) nsf_default_reference(h); return LBM_OK; }
        if (n == "mms_p0") { h->mms_p0 = v; if (!h->q0_set) nsf_default_reference(h); return LBM_OK; }
        if (n == "mms_u0") { h->mms_u0 = v; if (!h->q0_set) nsf_default_reference(h); return LBM_OK; }
        break;
    }
    return fail(h, LBM_EINVAL, "unknown parameter '" + n + "' for this system");
}

int lbm_get_param(const lbm_state *h, const char *name, double *v)
{
    if (!h || !name || !v) return LBM_EINVAL;
    const std::string n(name);
    const double lam = h->dt / h->dx;
    if (n == "dt") *v = h->dt;
    else if (n == "dx") *v = h->dx;
    else if (n == "lambda") *v = lam;
    else if (n == "tau") *v = h->tau;
    else if (n == "omega") *v = h->bound ? h->omega_c : 1.0 / h->tau;
    else if (n == "omega_tracker") *v = h->bound ? h->omega_t : (h->g_tau > 0 ? 1.0 / (h->g_tau + 1.0) : 0.0);
    else if (n == "trt_lambda") *v = h->trt_lambda;
    else if (n == "regularized") *v = h->regularized ? 1.0 : 0.0;
    else if (n == "omega_plus" || n == "omega_plus_tracker") {
        const int c = n == "omega_plus" ? 0 : 1;
        if (!h->bound) return LBM_EINVAL;                  // defined once bound
        *v = h->trt_lambda > 0 ? h->trt_a[c] + h->trt_b[c] : (c ? h->omega_t : h->omega_c);
    }
    else if (n == "tau_grad") *v = h->g_tau > 0 ? h->g_tau * h->dt : 0.0;
    else if (n == "g_tau") *v = h->g_tau;
    else if (n == "g") *v = h->g;
    else if (n == "t0") *v = h->t0;
    else if (n == "check_every") *v = (double)h->check_every;
    else if (n == "graphs") *v = h->use_graphs ? 1.0 : 0.0;
    else return LBM_EINVAL;
    return LBM_OK;
}

int lbm_set_storage(lbm_state *h, int storage)
{
    if (!h) return LBM_EINVAL;
    if (h->bound) return fail(h, LBM_EINVAL, "storage is fixed once bound");
    if (storage < LBM_F64 || storage > LBM_F16NE) return fail(h, LBM_EINVAL, "unknown storage");
    h->storage = storage;
    return LBM_OK;
}

int lbm_set_reference(lbm_state *h, const double *Q0)
{
    if (!h || !Q0) return LBM_EINVAL;
    if (h->bound) return fail(h, LBM_EINVAL, "reference is fixed once bound");
    for (int k = 0; k < h->K; ++k)
        if (!std::isfinite(Q0[k])) return fail(h, LBM_EINVAL, "reference state is not finite");
    if (h->sys == SYS_HCNSF)
        for (int k = 5; k < h->K; ++k)
            if (Q0[k] != 0.0) return fail(h, LBM_EINVAL, "hcnsf3d_trk14: the reference trackers must be zero");
    if (h->sys >= SYS_GEN0)
        for (int k = gen_conserved(h->sys); k < h->K; ++k)
            if (Q0[k] != 0.0) return fail(h, LBM_EINVAL, "generated systems: the reference trackers must be zero");
    for (int k = 0; k < h->K; ++k) h->Q0[k] = Q0[k];
    h->q0_set = true;
    return LBM_OK;
}

int lbm_get_reference(const lbm_state *h, double *Q0_out)
{
    if (!h || !Q0_out) return LBM_EINVAL;
    for (int k = 0; k < h->K; ++k) Q0_out[k] = h->storage == LBM_F64 ? h->Q0[k] : (double)(float)h->Q0[k];
    return LBM_OK;
}

size_t lbm_required_bytes(const lbm_state *h, int which)
{
    if (!h) return 0;
    if (which == 0) {
        if (h->storage == LBM_F16NE)   // binary16 deviations (tile-blocked, padded), then FP32 moments
            return ((((size_t)h->K * h->Q * (size_t)padded_plane(h->C) * 2) + 255) & ~(size_t)255) +
                   (size_t)h->K * h->C * 4;
        // tile-blocked [nz][tiles][K][Q][kTile], each slab padded to whole tiles
        const size_t s = h->storage == LBM_F64 ? 8 : (h->storage == LBM_F32 ? 4 : 2);
        return (size_t)h->K * h->Q * (size_t)padded_plane((long long)h->nx * h->ny) * (size_t)h->nz * s;
    }
    if (which == 1) return aux_bytes();
    return 0;
}

int lbm_bind(lbm_state *h, void *pop_a, void *pop_b, void *aux, void *hip_stream)
{
    if (!h) return LBM_EINVAL;
    if (h->bound) return fail(h, LBM_EINVAL, "already bound");
    if (!pop_a || !pop_b || !aux || pop_a == pop_b) return fail(h, LBM_EINVAL, "need two distinct population buffers and a scratch buffer");
    if (((uintptr_t)pop_a | (uintptr_t)pop_b | (uintptr_t)aux) & 255u)
        return fail(h, LBM_EINVAL, "buffers must be 256-byte aligned");
    if (has_trackers(h->sys) && !(h->g_tau > 0)) return fail(h, LBM_EINVAL, "set g_tau before binding");
    if (h->storage == LBM_F16NE && h->field_src) return fail(h, LBM_EINVAL, "no explicit source field with F16NE storage");
    h->L = lbm_launchers(h->sys, h->lat, h->storage);
    if (!h->L) return fail(h, LBM_EINVAL, "no kernel for this system, lattice and storage");
    // Parameters in use.  With single-precision arithmetic the kernels see
    // dt/dx rounded once to float and 2 - omega on the 2^-24 grid; the handle keeps the
    // values those roundings define (dt = float(dt/dx) dx, omega = 2 -
    // float(2 - omega)) so that time, diagnostics and lbm_get_param describe
    // exactly the scheme that runs.
    h->omega_c = 1.0 / h->tau;
    h->omega_t = has_trackers(h->sys) ? 1.0 / (h->g_tau + 1.0) : h->omega_c;
    if (h->storage != LBM_F64) {
        for (int k = 0; k < h->K; ++k) h->Q0[k] = (double)(float)h->Q0[k];
        h->dt = (double)(float)(h->dt / h->dx) * h->dx;
        // 2 - omega on the 2^-24 grid, so that omega - 1 and 2 - omega are
        // both exact in float (a change of tau - 1/2 below 1e-5 relative)
        h->omega_c = 2.0 - std::nearbyint((2.0 - h->omega_c) * 16777216.0) / 16777216.0;
        h->omega_t = 2.0 - std::nearbyint((2.0 - h->omega_t) * 16777216.0) / 16777216.0;
        h->tau = 1.0 / h->omega_c;
    }
    if (h->regularized && (h->trt_lambda > 0 || h->storage == LBM_F16NE))
        return fail(h, LBM_EINVAL, "the regularized collision excludes trt_lambda and F16NE storage");
    if (h->trt_lambda > 0) {
        if (h->storage == LBM_F16NE) return fail(h, LBM_EINVAL, "two-relaxation-time collision needs F64/F32/F16 storage");
        // omega- is the BGK rate (the flux moment relaxes at it); omega+ from
        // the magic parameter.  The kernels use a = (omega+ + omega-)/2 and
        // b = (omega+ - omega-)/2; in single precision 2 - a sits on the 2^-24
        // grid (a - 1 exact) and b is rounded once, and the rates in use are
        // a -+ b.
        double *om[2] = {&h->omega_c, &h->omega_t};
        for (int c = 0; c < 2; ++c) {
            const double wm = *om[c];
            const double wp = 1.0 / (0.5 + h->trt_lambda / (1.0 / wm - 0.5));
            double a = 0.5 * (wp + wm), b = 0.5 * (wp - wm);
            if (h->storage != LBM_F64) {
                a = 2.0 - std::nearbyint((2.0 - a) * 16777216.0) / 16777216.0;
                b = (double)(float)b;
            }
            h->trt_a[c] = a;
            h->trt_b[c] = b;
            *om[c] = a - b;
        }
        if (!has_trackers(h->sys)) {
            h->trt_a[1] = h->trt_a[0];
            h->trt_b[1] = h->trt_b[0];
            h->omega_t = h->omega_c;
        }
        h->tau = 1.0 / h->omega_c;
    }
    h->pop[0] = pop_a;
    h->pop[1] = pop_b;
    h->cur = 0;
    h->aux = aux;
    h->stream = (hipStream_t)hip_stream;
    h->bound = true;
    return LBM_OK;
}

int lbm_set_field(lbm_state *h, const char *name, const void *dev_ptr)
{
    if (!h || !name) return LBM_EINVAL;
    // kernels read a field through its pointer: captured launches stay valid
    // while the pointer does (the contents may change between steps)
    auto attach = [h](const void *&slot, const void *ptr) {
        if (slot != ptr) h->epoch += 1;
        slot = ptr;
        return LBM_OK;
    };
    if (h->sys == SYS_SWE && !std::strcmp(name, "grad_zb")) return attach(h->field_b, dev_ptr);
    if (!std::strcmp(name, "source")) {
        if (h->storage == LBM_F16NE) return fail(h, LBM_EINVAL, "no explicit source field with F16NE storage");
        return attach(h->field_src, dev_ptr);
    }
    if (h->sys == SYS_HCNSF && !std::strcmp(name, "coef")) {
        if (h->storage == LBM_F16NE) return fail(h, LBM_EINVAL, "no coefficient field with F16NE storage");
        return attach(h->field_b, dev_ptr);
    }
    return fail(h, LBM_EINVAL, std::string("unknown field '") + name + "' for this system");
}

int lbm_reduce(lbm_state *h, int what, const double *ref_dev, double *host_out);

int lbm_init_moments(lbm_state *h, const double *Q_dev)
{
    int rc = check_ready(h);
    if (rc) return rc;
    if (!Q_dev) return fail(h, LBM_EINVAL, "null field pointer");
    hipError_t e;
    for (int k = 0; k < LBM_MAXK; ++k) h->scale_exp[k] = 0;
    if (h->storage == LBM_F16 || h->storage == LBM_F16NE) {
        // per-field power-of-two scale: the largest initial stored magnitude
        // maps near 2^11 (binary16 holds up to 65504)
        e = h->L->init_absmax(*h, Q_dev, (double *)h->aux, h->stream);
        if (e != hipSuccess) return hipfail(h, e, "init_absmax");
        std::vector<double> part((size_t)h->K * kRedBlocks);
        e = hipMemcpyAsync(part.data(), h->aux, part.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hipfail(h, e, "init_absmax copy");
        for (int k = 0; k < h->K; ++k) {
            double m = 0.0;
            for (int b = 0; b < kRedBlocks; ++b) m = std::fmax(m, part[(size_t)k * kRedBlocks + b]);
            int ex = 0;
            if (m > 0.0 && std::isfinite(m)) ex = (int)std::floor(std::log2(2048.0 / m));
            h->scale_exp[k] = ex < -24 ? -24 : (ex > 24 ? 24 : ex);
        }
    }
    h->cur = 0;
    h->nsteps = 0;
    h->epoch += 1;                      // the F16 scales may have changed
    e = h->L->init(*h, Q_dev, h->pop[0], h->stream);
    if (e != hipSuccess) return hipfail(h, e, "init");
    if (h->check_subchar) {
        double sp[2];
        rc = lbm_reduce(h, LBM_RED_MAXSPEED, nullptr, sp);
        if (rc) return rc;
        if (!(sp[1] <= 1.0)) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "sub-characteristic bound violated: (dt/dx) max|eig A_n| = %.6g > cs = %.6g",
                          sp[0], std::sqrt(h->cs2));
            return fail(h, LBM_ESUBCHAR, buf);
        }
    }
    return LBM_OK;
}

// Failure detection (Sec. 2.4.2: outside the sub-characteristic bound the
// scheme blows up): with check_every = N > 0, after every step whose count
// is a multiple of N the populations are scanned for non-finite values (the
// LBM_RED_NONFINITE reduction, which synchronises) and stepping stops there.
static int check_finite(lbm_state *h)
{
    double cnt = 0.0;
    const int rc = lbm_reduce(h, LBM_RED_NONFINITE, nullptr, &cnt);
    if (rc) return rc;
    if (cnt != 0.0) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "%.0f non-finite populations after step %lld", cnt, h->nsteps);
        return fail(h, LBM_ENONFINITE, buf);
    }
    return LBM_OK;
}

static int run_steps(lbm_state *h, int n, void *qhist)
{
    int rc = check_ready(h);
    if (rc) return rc;
    if (n < 0) return fail(h, LBM_EINVAL, "negative step count");
    const size_t stride = (size_t)h->K * (size_t)h->C * arith_bytes(h);
    int j = 0;
    if (batch_launches(h, n)) {
        for (int len; (len = std::min(kGraphChunk, n - j)) >= kGraphMinLaunches; j += len) {
            char *q0 = qhist ? (char *)qhist + (size_t)j * stride : nullptr;
            const GraphKey key = {0, len, h->cur, h->epoch, {h->pop[0], h->pop[1], q0, nullptr}};
            const int cur0 = h->cur;
            rc = replay(h, key, [&](hipStream_t s) {
                int c = cur0;
                for (int i = 0; i < len; ++i) {
                    const hipError_t e = h->L->step(*h, h->pop[c], h->pop[c ^ 1], q0 ? q0 + (size_t)i * stride : nullptr, s);
                    if (e != hipSuccess) return e;
                    c ^= 1;
                }
                return hipSuccess;
            });
            if (rc) return rc;
            h->cur ^= len & 1;
            h->nsteps += len;
        }
    }
    for (; j < n; ++j) {
        void *q = qhist ? (char *)qhist + (size_t)j * stride : nullptr;
        const hipError_t e = h->L->step(*h, h->pop[h->cur], h->pop[h->cur ^ 1], q, h->stream);
        if (e != hipSuccess) return hipfail(h, e, "step");
        h->cur ^= 1;
        h->nsteps += 1;
        if (h->check_every > 0 && h->nsteps % h->check_every == 0) {
            rc = check_finite(h);
            if (rc) return rc;
        }
    }
    return LBM_OK;
}

int lbm_step(lbm_state *h, int n) { return run_steps(h, n, nullptr); }

int lbm_step_record(lbm_state *h, int n, void *Q_hist_dev)
{
    if (h && !Q_hist_dev) return fail(h, LBM_EINVAL, "null history pointer");
    if (h && h->storage == LBM_F16NE) return fail(h, LBM_EINVAL, "no moment history with F16NE storage");
    if (h && (h->trt_lambda > 0 || h->regularized))
        return fail(h, LBM_EINVAL, "the moment history and the adjoint are BGK only");
    return run_steps(h, n, Q_hist_dev);
}

int lbm_moments(lbm_state *h, void *Q_out_dev, int absolute, int out_dtype)
{
    int rc = check_ready(h);
    if (rc) return rc;
    if (!Q_out_dev || (out_dtype != LBM_F64 && out_dtype != LBM_F32)) return fail(h, LBM_EINVAL, "bad output");
    const hipError_t e = h->L->moments(*h, h->pop[h->cur], Q_out_dev, absolute, out_dtype == LBM_F64 ? 0 : 1, h->stream);
    return e == hipSuccess ? LBM_OK : hipfail(h, e, "moments");
}

// The two reduction passes with workspace ws: partial results of the first
// pass ([slot][block]) and the final slots after them.
static int reduce_with(lbm_state *h, int what, const double *ref_dev, double *host_out, double *ws)
{
    int rc = check_ready(h);
    if (rc) return rc;
    if (!host_out || what < LBM_RED_SUMS || what > LBM_RED_NONFINITE) return fail(h, LBM_EINVAL, "bad reduction");
    if ((what == LBM_RED_RELL2 || what == LBM_RED_RELLINF) && !ref_dev) return fail(h, LBM_EINVAL, "reference field required");
    hipError_t e = h->L->reduce(*h, h->pop[h->cur], what, ref_dev, ws, h->stream);
    if (e != hipSuccess) return hipfail(h, e, "reduce");
    const int nslot = (what == LBM_RED_MAXSPEED || what == LBM_RED_NONFINITE) ? 1 : (what == LBM_RED_SUMS ? h->K : 2 * h->K);
    double r[2 * LBM_MAXK];
    e = hipMemcpyAsync(r, ws + (size_t)2 * LBM_MAXK * kRedBlocks, nslot * sizeof(double), hipMemcpyDeviceToHost,
                       h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hipfail(h, e, "reduce copy");
    switch (what) {
    case LBM_RED_SUMS:
        for (int k = 0; k < h->K; ++k) host_out[k] = r[k];
        break;
    case LBM_RED_RELL2:
        for (int k = 0; k < h->K; ++k) host_out[k] = r[h->K + k] > 0 ? std::sqrt(r[k] / r[h->K + k]) : std::sqrt(r[k]);
        break;
    case LBM_RED_RELLINF:
        for (int k = 0; k < h->K; ++k) host_out[k] = r[h->K + k] > 0 ? r[k] / r[h->K + k] : r[k];
        break;
    case LBM_RED_MAXSPEED:
        host_out[0] = (h->dt / h->dx) * r[0];
        host_out[1] = host_out[0] / std::sqrt(h->cs2);
        break;
    case LBM_RED_NONFINITE:
        host_out[0] = r[0];
        break;
    }
    return LBM_OK;
}

int lbm_reduce(lbm_state *h, int what, const double *ref_dev, double *host_out)
{
    return reduce_with(h, what, ref_dev, host_out, h ? (double *)h->aux : nullptr);
}

// Reduction workspace of lbm_reduce_static: one array per GPU, in device
// memory the code object reserves when it is loaded, so the entry point
// allocates nothing.  Host code reaches it only through the address
// hipGetSymbolAddress returns on each device (the array's name is a host
// stand-in, not a device address).
constexpr size_t kStaticScratchDoubles = (size_t)2 * LBM_MAXK * kRedBlocks + 4 * LBM_MAXK;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

// address of this device's scratch array, looked up once per device with
// that device current
double *static_scratch(lbm_state *h, int *rc)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *rc = hipfail(h, e, "reduce_static: hipGetDevice");
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        *rc = fail(h, LBM_EINVAL, "reduce_static: device index beyond the library's table");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *rc = hipfail(h, e != hipSuccess ? e : hipErrorInvalidSymbol, "reduce_static: hipGetSymbolAddress");
            return nullptr;
        }
        g_scratch_ptr[dev] = (double *)p;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

int lbm_reduce_static(lbm_state *h, int what, const double *ref_dev, double *host_out)
{
    int rc = check_ready(h);
    if (rc) return rc;
    // the passes need 2 K partial slots per first-pass workgroup and the
    // final slots after the partials of the largest system
    const size_t need = (size_t)2 * h->K * kRedBlocks;
    if (h->K > LBM_MAXK || need + 2 * LBM_MAXK > kStaticScratchDoubles)
        return fail(h, LBM_EINVAL, "reduce_static: the reduction needs more than the static workspace of " +
                                       std::to_string(kStaticScratchDoubles * sizeof(double)) + " bytes");
    double *ws = static_scratch(h, &rc);
    if (!ws) return rc;
    return reduce_with(h, what, ref_dev, host_out, ws);
}

long long lbm_step_count(const lbm_state *h) { return h ? h->nsteps : 0; }
double lbm_time(const lbm_state *h) { return h ? h->t0 + h->nsteps * h->dt : 0.0; }

int lbm_adjoint_seed(lbm_state *h, const void *dLdQ_dev, void *lam_dev)
{
    int rc = check_ready(h);
    if (rc) return rc;
    if (h->trt_lambda > 0 || h->regularized) return fail(h, LBM_EINVAL, "the adjoint is BGK only");
    if (!h->L->adj_seed) return fail(h, LBM_EINVAL, "no adjoint for this system");
    if (!dLdQ_dev || !lam_dev) return fail(h, LBM_EINVAL, "null pointer");
    const hipError_t e = h->L->adj_seed(*h, dLdQ_dev, lam_dev, h->stream);
    return e == hipSuccess ? LBM_OK : hipfail(h, e, "adjoint_seed");
}

int lbm_adjoint_step(lbm_state *h, int n, void *lam_a, void *lam_b, const void *Q_hist_dev, void *grad_field_dev)
{
    int rc = check_ready(h);
    if (rc) return rc;
    if (h->trt_lambda > 0 || h->regularized) return fail(h, LBM_EINVAL, "the adjoint is BGK only");
    if (!h->L->adj_step) return fail(h, LBM_EINVAL, "no adjoint for this system");
    if (n < 0 || !lam_a || !lam_b || lam_a == lam_b || (n > 0 && !Q_hist_dev)) return fail(h, LBM_EINVAL, "bad adjoint arguments");
    if (grad_field_dev && !h->field_b) return fail(h, LBM_EINVAL, "no source field attached");
    const size_t stride = (size_t)h->K * (size_t)h->C * arith_bytes(h);
    void *in = lam_a, *out = lam_b;
    int j = n - 1;                       // next history slice, taken in reverse
    if (batch_launches(h, n)) {
        for (int len; (len = std::min(kGraphChunk, j + 1)) >= kGraphMinLaunches; j -= len) {
            const char *qtop = (const char *)Q_hist_dev + (size_t)j * stride;
            const GraphKey key = {1, len, 0, h->epoch, {in, out, qtop, grad_field_dev}};
            void *a = in, *b = out;
            rc = replay(h, key, [&](hipStream_t s) {
                void *x = a, *y = b;
                for (int i = 0; i < len; ++i) {
                    const hipError_t e = h->L->adj_step(*h, x, y, qtop - (size_t)i * stride, grad_field_dev, s);
                    if (e != hipSuccess) return e;
                    std::swap(x, y);
                }
                return hipSuccess;
            });
            if (rc) return rc;
            if (len & 1) std::swap(in, out);
        }
    }
    for (; j >= 0; --j) {
        const hipError_t e = h->L->adj_step(*h, in, out, (const char *)Q_hist_dev + (size_t)j * stride, grad_field_dev,
                                            h->stream);
        if (e != hipSuccess) return hipfail(h, e, "adjoint_step");
        void *t = in;
        in = out;
        out = t;
    }
    return LBM_OK;
}

int lbm_adjoint_to_initial(lbm_state *h, const void *lam0_dev, const double *Q_init_dev, double *dLdQ0_dev)
{
    int rc = check_ready(h);
    if (rc) return rc;
    if (h->trt_lambda > 0 || h->regularized) return fail(h, LBM_EINVAL, "the adjoint is BGK only");
    if (!h->L->adj_init) return fail(h, LBM_EINVAL, "no adjoint for this system");
    if (!lam0_dev || !Q_init_dev || !dLdQ0_dev) return fail(h, LBM_EINVAL, "null pointer");
    const hipError_t e = h->L->adj_init(*h, lam0_dev, Q_init_dev, dLdQ0_dev, h->stream);
    return e == hipSuccess ? LBM_OK : hipfail(h, e, "adjoint_to_initial");
}

int lbm_save(lbm_state *h, void *host_buf, size_t *n_inout)
{
    int rc = check_ready(h);
    if (rc) return rc;
    if (!n_inout) return fail(h, LBM_EINVAL, "null size pointer");
    const size_t payload = lbm_required_bytes(h, 0);
    const size_t need = sizeof(SaveHeader) + payload;
    if (!host_buf) {
        *n_inout = need;
        return LBM_OK;
    }
    if (*n_inout < need) return fail(h, LBM_EINVAL, "checkpoint buffer too small");
    SaveHeader hd;
    std::memset(&hd, 0, sizeof hd);
    std::memcpy(hd.magic, "LBMCKPT1", 8);
    hd.version = 2;                       // 2: per-field header arrays of 18 entries
    hd.sys = h->sys;
    hd.lat = h->lat;
    hd.storage = h->storage;
    hd.nx = h->nx;
    hd.ny = h->ny;
    hd.nz = h->nz;
    hd.K = h->K;
    hd.Q = h->Q;
    hd.nsteps = h->nsteps;
    hd.t0 = h->t0;
    hd.tau = h->tau;
    hd.dt = h->dt;
    hd.dx = h->dx;
    for (int k = 0; k < LBM_MAXK; ++k) {
        hd.Q0[k] = h->Q0[k];
        hd.scale_exp[k] = h->scale_exp[k];
    }
    hd.payload = payload;
    std::memcpy(host_buf, &hd, sizeof hd);
    hipError_t e = hipMemcpyAsync((char *)host_buf + sizeof hd, h->pop[h->cur], payload, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hipfail(h, e, "save");
    *n_inout = need;
    return LBM_OK;
}

int lbm_load(lbm_state *h, const void *host_buf, size_t n)
{
    int rc = check_ready(h);
    if (rc) return rc;
    if (!host_buf || n < sizeof(SaveHeader)) return fail(h, LBM_EINVAL, "checkpoint buffer too small");
    SaveHeader hd;
    std::memcpy(&hd, host_buf, sizeof hd);
    if (std::memcmp(hd.magic, "LBMCKPT1", 8) != 0 || hd.version != 2) return fail(h, LBM_EINVAL, "not a checkpoint of this version");
    if (hd.sys != h->sys || hd.lat != h->lat || hd.storage != h->storage || hd.nx != h->nx || hd.ny != h->ny ||
        hd.nz != h->nz)
        return fail(h, LBM_EINVAL, "checkpoint does not match this handle");
    const size_t payload = lbm_required_bytes(h, 0);
    if (hd.payload != payload || n < sizeof hd + payload) return fail(h, LBM_EINVAL, "checkpoint size mismatch");
    for (int k = 0; k < h->K; ++k)
        if (hd.Q0[k] != h->Q0[k]) return fail(h, LBM_EINVAL, "checkpoint reference state differs");
    for (int k = 0; k < LBM_MAXK; ++k) h->scale_exp[k] = hd.scale_exp[k];
    h->epoch += 1;
    h->nsteps = hd.nsteps;
    h->t0 = hd.t0;
    h->cur = 0;
    hipError_t e = hipMemcpyAsync(h->pop[0], (const char *)host_buf + sizeof hd, payload, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hipfail(h, e, "load");
    return LBM_OK;
}

int lbm_snapshot(lbm_state *h, void *dev_buf)
{
    int rc = check_ready(h);
    if (rc) return rc;
    if (!dev_buf) return fail(h, LBM_EINVAL, "null snapshot buffer");
    const hipError_t e = lbm_launch_copy(dev_buf, h->pop[h->cur], lbm_required_bytes(h, 0), h->stream);
    return e == hipSuccess ? LBM_OK : hipfail(h, e, "snapshot");
}

int lbm_restore(lbm_state *h, const void *dev_buf, long long step)
{
    int rc = check_ready(h);
    if (rc) return rc;
    if (!dev_buf || step < 0) return fail(h, LBM_EINVAL, "bad restore arguments");
    const hipError_t e = lbm_launch_copy(h->pop[h->cur], dev_buf, lbm_required_bytes(h, 0), h->stream);
    if (e != hipSuccess) return hipfail(h, e, "restore");
    h->nsteps = step;
    return LBM_OK;
}

int lbm_bw_copy(void *dst, const void *src, size_t n, void *hip_stream)
{
    if (!dst || !src) return LBM_EINVAL;
    return lbm_launch_copy(dst, src, n, (hipStream_t)hip_stream) == hipSuccess ? LBM_OK : LBM_EHIP;
}

int lbm_bw_streams(void *dst, const void *src, int nx, int ny, int fields, void *hip_stream)
{
    if (!dst || !src || nx < 1 || ny < 1 || (fields != 3 && fields != 6)) return LBM_EINVAL;
    return lbm_launch_streams(dst, src, nx, ny, fields, (hipStream_t)hip_stream) == hipSuccess ? LBM_OK : LBM_EHIP;
}

int lbm_bw_streams3(void *dst, const void *src, int nx, int ny, int nz, int fields, void *hip_stream)
{
    if (!dst || !src || nx < 1 || ny < 1 || nz < 1 || (fields != 14 && fields != 17)) return LBM_EINVAL;
    const hipError_t e = lbm_launch_streams3(dst, src, nx, ny, nz, fields, (hipStream_t)hip_stream);
    if (e == hipErrorInvalidValue) return LBM_EINVAL;
    return e == hipSuccess ? LBM_OK : LBM_EHIP;
}

void lbm_destroy(lbm_state *h)
{
    if (h && h->graphs) delete (GraphCache *)h->graphs;
    delete h;
}

}  // extern "C"
