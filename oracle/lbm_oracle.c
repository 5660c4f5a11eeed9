/* lbm_oracle.c -- plain FP64 CPU oracle of the per-field, exact-flux-
 * equilibrium BGK collide-and-stream scheme of
 *   Kummerlaender, Bukreev, Krause, "Automated Derivation of Lattice
 *   Boltzmann Methods for Systems of Conservation Laws".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the HIP library is checked against.  Only tests/, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the library never
 * does, and it shares no code, header or table with the library.
 *
 * What it computes (each step in the paper's order and notation):
 *   lattices           Sec. 2.2 isotropy conditions; D2Q5/D3Q7 from the
 *                      supplement's stencil table; D2Q9 standard weights
 *   initialisation     populations at the (shifted) equilibrium of the given
 *                      fields (supplement, numerical configuration)
 *   moments            eq. (moments) plus the reference shift (Sec. 2.5.2)
 *   equilibrium        eq. (feq), shifted by f^eq(Q0, F0) (Sec. 2.5.2)
 *   collide-and-stream eq. (lbe_update): BGK relaxation, source w_i dt S,
 *                      then push to x + c_i with periodic wrap
 *   adjoint            transpose of one step's Jacobian; the per-cell
 *                      (KQ x KQ) Jacobian is formed column by column with
 *                      complex-step differentiation (Squire & Trapp 1998),
 *                      which is exact to rounding for these analytic maps.
 * All arithmetic is IEEE double; build with -ffp-contract=off.
 */
#include <complex.h>
#include <omp.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXK 18
#define MAXQ 9

enum { SYS_ADVDIFF = 0, SYS_SWE = 1, SYS_NEOHOOKE = 2, SYS_NSF17 = 3, SYS_BURGERS = 4, SYS_EULER = 5,
       SYS_MAXWELL = 6, SYS_ALLENCAHN = 7, SYS_RELHYDRO = 8, SYS_NSE = 9, SYS_CNSF2D = 10,
       SYS_MHD = 11, SYS_HCNSF = 12 };
enum { LAT_D2Q5 = 0, LAT_D2Q9 = 1, LAT_D3Q7 = 2 };
enum {
    P_G = 0, P_AX, P_AY, P_AZ, P_NU, P_R, P_TAUG, P_GAMMA, P_MU, P_KAPPA,
    P_RHO0, P_MUS, P_LAMS, P_CLIGHT, P_CSPHYS, P_RGAS, P_COUNT
};

typedef struct {
    int system, lattice;
    int nx, ny, nz;
    int shifted;          /* 1: store f* = f - f^eq(Q0, F0); 0: store f    */
    double lam;           /* dt / dx                                        */
    double dt;
    double omega[MAXK];   /* per-field collision rate                       */
    double Q0[MAXK];      /* reference state (zeros when unshifted)          */
    double par[16];       /* physical parameters, indices P_*                */
    int trt;              /* collision: 0 BGK, 1 two-relaxation-time,
                             2 regularized (first-order Hermite projection) */
    double omega_plus[MAXK]; /* TRT: rate of the symmetric parts; omega[] then
                                relaxes the antisymmetric parts              */
} oracle_cfg;

typedef struct {
    int D, Q;
    int c[MAXQ][3];
    double w[MAXQ];
    double cs2;
    int opp[MAXQ];        /* index of the opposite velocity -c_i            */
} lattice;

static lattice lattice_get(int id)
{
    lattice L;
    memset(&L, 0, sizeof L);
    if (id == LAT_D2Q5) {
        /* rest, +x, +y, -x, -y; w = 1/3, 1/6; cs^2 = 1/3 */
        static const int c[5][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}};
        L.D = 2; L.Q = 5; L.cs2 = 1.0 / 3.0;
        for (int i = 0; i < 5; ++i) {
            L.c[i][0] = c[i][0]; L.c[i][1] = c[i][1];
            L.w[i] = (i == 0) ? 1.0 / 3.0 : 1.0 / 6.0;
        }
    } else if (id == LAT_D2Q9) {
        /* rest, 4 axis, 4 diagonal; w = 4/9, 1/9, 1/36; cs^2 = 1/3 */
        static const int c[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1},
                                    {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
        L.D = 2; L.Q = 9; L.cs2 = 1.0 / 3.0;
        for (int i = 0; i < 9; ++i) {
            L.c[i][0] = c[i][0]; L.c[i][1] = c[i][1];
            L.w[i] = (i == 0) ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
        }
    } else {
        /* D3Q7: rest, +-x, +-y, +-z; w = 1/4, 1/8; cs^2 = 1/4 */
        static const int c[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                                    {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
        L.D = 3; L.Q = 7; L.cs2 = 1.0 / 4.0;
        for (int i = 0; i < 7; ++i) {
            for (int a = 0; a < 3; ++a) L.c[i][a] = c[i][a];
            L.w[i] = (i == 0) ? 1.0 / 4.0 : 1.0 / 8.0;
        }
    }
    for (int i = 0; i < L.Q; ++i)
        for (int j = 0; j < L.Q; ++j)
            if (L.c[j][0] == -L.c[i][0] && L.c[j][1] == -L.c[i][1] && L.c[j][2] == -L.c[i][2]) L.opp[i] = j;
    return L;
}

static int system_K(int sys)
{
    switch (sys) {
    case SYS_ADVDIFF: return 3;
    case SYS_SWE: return 3;
    case SYS_NEOHOOKE: return 6;
    case SYS_NSF17: return 17;
    case SYS_BURGERS: return 1;
    case SYS_EULER: return 4;
    case SYS_MAXWELL: return 3;
    case SYS_ALLENCAHN: return 3;
    case SYS_RELHYDRO: return 3;
    case SYS_NSE: return 7;
    case SYS_CNSF2D: return 12;
    case SYS_MHD: return 18;
    case SYS_HCNSF: return 14;
    }
    return 0;
}

/* Components of the per-cell coefficient field: the prescribed porosity and
 * solid velocity (alpha, u_s) of the homogenized NSF system, otherwise one
 * per dimension (SWE: grad z_b). */
static int system_nb(int sys, int D) { return sys == SYS_HCNSF ? 4 : D; }
#define MAXB 4

/* ---- scalar-type instantiations of the cell arithmetic ---- */
#define T double
#define FN(name) name##_re
#define LOG(x) log(x)
#define SQRT(x) sqrt(x)
#include "oracle_cell.inc"
#undef T
#undef FN
#undef LOG
#undef SQRT

#define T double complex
#define FN(name) name##_cx
#define LOG(x) clog(x)
#define SQRT(x) csqrt(x)
#include "oracle_cell.inc"
#undef T
#undef FN
#undef LOG
#undef SQRT

static void reference_flux(const oracle_cfg *cfg, int K, double *F0)
{
    double Phi[MAXK][3];
    memset(F0, 0, sizeof(double) * MAXK * 3);
    memset(Phi, 0, sizeof Phi);
    if (!cfg->shifted) return;
    flux_re(cfg->system, cfg->par, cfg->Q0, NULL, Phi);
    for (int k = 0; k < K; ++k)
        for (int a = 0; a < 3; ++a) F0[k * 3 + a] = Phi[k][a];
}

static inline long wrap(long v, long n) { return ((v % n) + n) % n; }

/* ------------------------------------------------------------------ API */

int oracle_num_fields(int sys) { return system_K(sys); }
int oracle_num_velocities(int lat) { return lattice_get(lat).Q; }

/* Physical flux Phi (K x 3, row-major) and source S (K) at one state Q;
 * b: the cell's coefficient values (system_nb of them) or NULL. */
void oracle_flux(const oracle_cfg *cfg, const double *Q, const double *b, double *Phi_out)
{
    double Phi[MAXK][3];
    memset(Phi, 0, sizeof Phi);
    flux_re(cfg->system, cfg->par, Q, b, Phi);
    const int K = system_K(cfg->system);
    for (int k = 0; k < K; ++k)
        for (int a = 0; a < 3; ++a) Phi_out[k * 3 + a] = Phi[k][a];
}

void oracle_source(const oracle_cfg *cfg, const double *Q, const double *b, double *S)
{
    source_re(cfg->system, cfg->par, Q, b, S);
}

/* Equilibrium initialisation: f*_{k,i}(x) = w_i [ (Q_k - Q0_k)
 *   + (lam/cs2) c_i . (Phi_k(Q) - F0_k) ] at every cell, from fields
 * Q[k*C + cell] (SoA) and the coefficient field (nb*C, may be NULL).
 * Output f[(k*Qn + i)*C + cell]. */
void oracle_init(const oracle_cfg *cfg, const double *Qf, const double *bfield, double *f)
{
    const lattice L = lattice_get(cfg->lattice);
    const int K = system_K(cfg->system);
    const long C = (long)cfg->nx * cfg->ny * cfg->nz;
    double F0[MAXK * 3];
    reference_flux(cfg, K, F0);
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < C; ++cell) {
        double Q[MAXK], Phi[MAXK][3], b[MAXB];
        memset(Phi, 0, sizeof Phi);
        for (int k = 0; k < K; ++k) Q[k] = Qf[k * C + cell];
        const int nb = system_nb(cfg->system, L.D);
        if (bfield)
            for (int a = 0; a < nb; ++a) b[a] = bfield[a * C + cell];
        flux_re(cfg->system, cfg->par, Q, bfield ? b : NULL, Phi);
        for (int k = 0; k < K; ++k)
            for (int i = 0; i < L.Q; ++i) {
                double cdot = 0.0;
                for (int a = 0; a < L.D; ++a)
                    cdot += L.c[i][a] * (Phi[k][a] - F0[k * 3 + a]);
                f[((long)k * L.Q + i) * C + cell] =
                    L.w[i] * ((Q[k] - cfg->Q0[k]) + (cfg->lam / L.cs2) * cdot);
            }
    }
}

/* Moments Q_k(x) = Q0_k + sum_i f*_{k,i}(x) (eq. moments, shifted). */
void oracle_moments(const oracle_cfg *cfg, const double *f, double *Qf)
{
    const lattice L = lattice_get(cfg->lattice);
    const int K = system_K(cfg->system);
    const long C = (long)cfg->nx * cfg->ny * cfg->nz;
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < C; ++cell)
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int i = 0; i < L.Q; ++i) s += f[((long)k * L.Q + i) * C + cell];
            Qf[k * C + cell] = cfg->Q0[k] + s;
        }
}

/* One collide-and-stream step (eq. lbe_update), push form:
 *   f_out_{k,i}(x + c_i mod N) = post_{k,i}(x).
 * S_ext (K*C, may be NULL): explicit source added to S_k, e.g. the
 * manufactured-solution forcing at t + dt/2.  b (nb*C, may be NULL):
 * per-cell coefficient field (SWE: grad z_b; homogenized NSF: alpha, u_s). */
void oracle_step(const oracle_cfg *cfg, const double *fin, double *fout,
                 const double *S_ext, const double *bfield)
{
    const lattice L = lattice_get(cfg->lattice);
    const int K = system_K(cfg->system);
    const long nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
    const long C = nx * ny * nz;
    double F0[MAXK * 3];
    reference_flux(cfg, K, F0);
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < C; ++cell) {
        const long x = cell % nx, y = (cell / nx) % ny, z = cell / (nx * ny);
        double f[MAXK * MAXQ], post[MAXK * MAXQ], Sx[MAXK], b[MAXB];
        for (int k = 0; k < K; ++k)
            for (int i = 0; i < L.Q; ++i) f[k * L.Q + i] = fin[((long)k * L.Q + i) * C + cell];
        if (S_ext)
            for (int k = 0; k < K; ++k) Sx[k] = S_ext[k * C + cell];
        if (bfield)
            for (int a = 0; a < system_nb(cfg->system, L.D); ++a) b[a] = bfield[a * C + cell];
        collide_cell_re(cfg, &L, K, F0, f, bfield ? b : NULL, S_ext ? Sx : NULL, post);
        for (int i = 0; i < L.Q; ++i) {
            const long xd = wrap(x + L.c[i][0], nx);
            const long yd = wrap(y + L.c[i][1], ny);
            const long zd = wrap(z + L.c[i][2], nz);
            const long dest = (zd * ny + yd) * nx + xd;
            for (int k = 0; k < K; ++k) fout[((long)k * L.Q + i) * C + dest] = post[k * L.Q + i];
        }
    }
}

/* Discrete adjoint of oracle_step.  With J(x) = d post(x) / d f(x) (the
 * cell's KQ x KQ collision Jacobian at the pre-collision populations f_n)
 * and mu_m(x) = lam_next_m(x + c_{i(m)}) the adjoint gathered back along
 * the streaming links,
 *   lam_out_n(x) = sum_m J_mn(x) mu_m(x).
 * If grad_b != NULL, also accumulates d L / d b_a(x) += sum_m mu_m(x)
 * d post_m(x) / d b_a(x).  Each Jacobian column is the imaginary part of
 * the collision evaluated at f + i h e_n, divided by h. */
void oracle_adjoint_step(const oracle_cfg *cfg, const double *lam_next, double *lam_out,
                         const double *f_n, const double *bfield, double *grad_b)
{
    const lattice L = lattice_get(cfg->lattice);
    const int K = system_K(cfg->system);
    const int KQ = K * L.Q;
    const long nx = cfg->nx, ny = cfg->ny, nz = cfg->nz;
    const long C = nx * ny * nz;
    const double h = 1e-30;
    double F0[MAXK * 3];
    reference_flux(cfg, K, F0);
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < C; ++cell) {
        const long x = cell % nx, y = (cell / nx) % ny, z = cell / (nx * ny);
        double complex f[MAXK * MAXQ], post[MAXK * MAXQ], b[MAXB];
        double mu[MAXK * MAXQ];
        for (int k = 0; k < K; ++k)
            for (int i = 0; i < L.Q; ++i) {
                f[k * L.Q + i] = f_n[((long)k * L.Q + i) * C + cell];
                const long xs = wrap(x + L.c[i][0], nx);
                const long ys = wrap(y + L.c[i][1], ny);
                const long zs = wrap(z + L.c[i][2], nz);
                mu[k * L.Q + i] = lam_next[((long)k * L.Q + i) * C + (zs * ny + ys) * nx + xs];
            }
        const int nb = system_nb(cfg->system, L.D);
        for (int a = 0; a < MAXB; ++a) b[a] = (bfield && a < nb) ? bfield[a * C + cell] : 0.0;
        for (int n = 0; n < KQ; ++n) {
            const double complex keep = f[n];
            f[n] = keep + I * h;
            collide_cell_cx(cfg, &L, K, F0, f, bfield ? b : NULL, NULL, post);
            f[n] = keep;
            double acc = 0.0;
            for (int m = 0; m < KQ; ++m) acc += (cimag(post[m]) / h) * mu[m];
            const int k = n / L.Q, i = n % L.Q;
            lam_out[((long)k * L.Q + i) * C + cell] = acc;
        }
        if (grad_b && bfield) {
            for (int a = 0; a < nb; ++a) {
                const double complex keep = b[a];
                b[a] = keep + I * h;
                collide_cell_cx(cfg, &L, K, F0, f, b, NULL, post);
                b[a] = keep;
                double acc = 0.0;
                for (int m = 0; m < KQ; ++m) acc += (cimag(post[m]) / h) * mu[m];
                grad_b[a * C + cell] += acc;
            }
        }
    }
}

/* d f*^0 / d Q^0 applied transposed: given lam0 = dL/df*^0 (K*Qn*C) and the
 * initial fields Q (K*C), returns dL/dQ^0 (K*C) through the equilibrium
 * initialisation, again column by column with complex steps. */
void oracle_init_adjoint(const oracle_cfg *cfg, const double *lam0, const double *Qf, double *dQ)
{
    const lattice L = lattice_get(cfg->lattice);
    const int K = system_K(cfg->system);
    const long C = (long)cfg->nx * cfg->ny * cfg->nz;
    const double h = 1e-30;
    double F0[MAXK * 3];
    reference_flux(cfg, K, F0);
#pragma omp parallel for schedule(static)
    for (long cell = 0; cell < C; ++cell) {
        double complex Q[MAXK], Phi[MAXK][3];
        for (int k = 0; k < K; ++k) Q[k] = Qf[k * C + cell];
        for (int m = 0; m < K; ++m) {
            const double complex keep = Q[m];
            Q[m] = keep + I * h;
            memset(Phi, 0, sizeof Phi);
            flux_cx(cfg->system, cfg->par, Q, NULL, Phi);
            double acc = 0.0;
            for (int k = 0; k < K; ++k)
                for (int i = 0; i < L.Q; ++i) {
                    double complex cdot = 0.0;
                    for (int a = 0; a < L.D; ++a) cdot += L.c[i][a] * (Phi[k][a] - F0[k * 3 + a]);
                    const double complex fe = L.w[i] * ((Q[k] - cfg->Q0[k]) + (cfg->lam / L.cs2) * cdot);
                    acc += (cimag(fe) / h) * lam0[((long)k * L.Q + i) * C + cell];
                }
            Q[m] = keep;
            dQ[m * C + cell] = acc;
        }
    }
}

/* The velocity set of a lattice: c (Q x 3 ints), w (Q), cs2; returns Q. */
int oracle_lattice(int lat, int *c, double *w, double *cs2)
{
    const lattice L = lattice_get(lat);
    for (int i = 0; i < L.Q; ++i) {
        for (int a = 0; a < 3; ++a) c[i * 3 + a] = L.c[i][a];
        w[i] = L.w[i];
    }
    *cs2 = L.cs2;
    return L.Q;
}

/* Number of OpenMP threads a parallel region of the oracle uses. */
int oracle_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}
