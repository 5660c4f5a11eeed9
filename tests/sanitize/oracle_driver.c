/* Exercises every entry point of the FP64 oracle (tests/test_oracle_sanitized.py
 * builds it with -fsanitize=address,undefined): every system on each lattice
 * of its dimension, small periodic grids with odd sizes, shifted and
 * unshifted storage, BGK / TRT / regularized collisions, the explicit source
 * and coefficient fields, and the adjoint entry points.  The values are
 * arbitrary but finite; what is checked is that no access leaves its buffer
 * and no operation is undefined.  Prints "ok" and exits 0 on completion. */
#include <stdio.h>

#include "lbm_oracle.c"

static double frand(unsigned *s)
{
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / 16777216.0;      /* [0, 1) */
}

static int run(int sys, int lat, int nx, int ny, int nz, int shifted, int trt, unsigned seed)
{
    const lattice L = lattice_get(lat);
    const int K = system_K(sys);
    const long C = (long)nx * ny * nz;
    const int nb = system_nb(sys, L.D);
    oracle_cfg cfg;
    memset(&cfg, 0, sizeof cfg);
    cfg.system = sys;
    cfg.lattice = lat;
    cfg.nx = nx;
    cfg.ny = ny;
    cfg.nz = nz;
    cfg.shifted = shifted;
    cfg.lam = 0.05;
    cfg.dt = 1e-3;
    cfg.trt = trt;
    for (int k = 0; k < MAXK; ++k) {
        cfg.omega[k] = 1.6;
        cfg.omega_plus[k] = 1.2;
    }
    /* a positive background: densities, depths, deformation diagonals and
     * energies away from zero */
    for (int k = 0; k < K; ++k) cfg.Q0[k] = shifted ? 1.0 + 0.5 * k : 0.0;
    for (int p = 0; p < P_COUNT; ++p) cfg.par[p] = 0.1 + 0.05 * p;
    cfg.par[P_GAMMA] = 1.4;
    cfg.par[P_RHO0] = 1.0;
    cfg.par[P_TAUG] = 3e-3;

    double *Qf = malloc(sizeof(double) * K * C), *Qo = malloc(sizeof(double) * K * C);
    double *f = malloc(sizeof(double) * K * L.Q * C), *g = malloc(sizeof(double) * K * L.Q * C);
    double *lam = malloc(sizeof(double) * K * L.Q * C), *lam2 = malloc(sizeof(double) * K * L.Q * C);
    double *S = malloc(sizeof(double) * K * C), *b = malloc(sizeof(double) * nb * C);
    double *gb = calloc((size_t)nb * C, sizeof(double)), *dQ = malloc(sizeof(double) * K * C);
    double Phi[MAXK * 3], Sk[MAXK], Q1[MAXK], b1[MAXB];
    if (!Qf || !Qo || !f || !g || !lam || !lam2 || !S || !b || !gb || !dQ) return 1;
    for (long j = 0; j < K * C; ++j) Qf[j] = 1.0 + 0.5 * (j / C) + 0.05 * frand(&seed);
    for (long j = 0; j < K * C; ++j) S[j] = 0.01 * (frand(&seed) - 0.5);
    for (long j = 0; j < nb * C; ++j) b[j] = 0.2 + 0.6 * frand(&seed);
    for (long j = 0; j < K * L.Q * C; ++j) lam[j] = frand(&seed) - 0.5;
    for (int k = 0; k < K; ++k) Q1[k] = Qf[k * C];
    for (int a = 0; a < MAXB; ++a) b1[a] = 0.5;

    oracle_flux(&cfg, Q1, b1, Phi);
    oracle_source(&cfg, Q1, b1, Sk);
    oracle_init(&cfg, Qf, b, f);
    oracle_step(&cfg, f, g, S, b);
    oracle_step(&cfg, g, f, NULL, NULL);
    oracle_moments(&cfg, f, Qo);
    if (trt == 0 && K <= 6) {
        oracle_adjoint_step(&cfg, lam, lam2, f, b, gb);
        oracle_adjoint_step(&cfg, lam2, lam, g, NULL, NULL);
        oracle_init_adjoint(&cfg, lam, Qf, dQ);
    }
    free(Qf); free(Qo); free(f); free(g); free(lam); free(lam2); free(S); free(b); free(gb); free(dQ);
    return 0;
}

int main(void)
{
    static const int dims[] = {2, 2, 2, 3, 2, 2, 2, 2, 2, 2, 2, 2, 3};
    int cases = 0;
    for (int sys = 0; sys <= SYS_HCNSF; ++sys)
        for (int lat = 0; lat <= LAT_D3Q7; ++lat) {
            if ((lat == LAT_D3Q7) != (dims[sys] == 3)) continue;
            for (int trt = 0; trt <= 2; ++trt) {
                const int nz = dims[sys] == 3 ? 3 : 1;
                if (run(sys, lat, 5, 4, nz, 1, trt, 17u + sys) || run(sys, lat, 3, 7, nz, trt == 0 ? 0 : 1, trt, 5u))
                    return 2;
                cases += 2;
            }
        }
    int c[MAXQ * 3];
    double w[MAXQ], cs2;
    for (int lat = 0; lat <= LAT_D3Q7; ++lat) oracle_lattice(lat, c, w, &cs2);
    printf("ok %d cases, %d threads\n", cases, oracle_num_threads());
    return 0;
}
