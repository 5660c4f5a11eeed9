// Conservation-law systems of the collide-and-stream library: the flux
// Phi(Q) (K x D) and source S(Q) of d_t Q + div Phi = S (eq. pde_target)
// for each supported system, as device functors.
//
// Fluxes are written in fluctuation form: flux_delta returns
// dPhi = Phi(Q0 + dQ) - Phi(Q0) computed from the reference state and the
// deviation without ever forming Phi(Q) and Phi(Q0) separately, so that in
// single precision no large-minus-large cancellation occurs (the reason for
// the paper's reference and equilibrium shift, Sec. 2.5.2).  Each functor is
// a template over the scalar type S (float, double, or Dual<> for the
// adjoint's Jacobian contractions); reference data and parameters are in the
// arithmetic type R.
#pragma once

#include "dual.hpp"

#include <type_traits>

#define LBM_MAXK 18

// Per-run constants shared by all systems (filled on the host in double and
// converted to the arithmetic type R).
template <class R>
struct Phys {
    R Q0[LBM_MAXK];       // reference state
    R g;                  // SWE gravity
    R mm0_h0[3];          // SWE, Euler: m0_a m0_b / h0 (rho0) for (x,x), (x,y), (y,y)
    R Hu_ref[3];          // Euler: H0 u0_a, H0 = E0 + p0
    R a[3], nu, react;    // advection velocity, diffusivity, reaction rate
    R inv_tau_grad;       // 1 / tau_grad, tau_grad = g_tau dt
    R gamma, mu, kappa;   // NSF
    R u_ref[3];           // reference velocity m0 / rho0
    R p_ref, T_ref, H_ref;// reference pressure, temperature p0/rho0, E0 + p0
    R tau_ref[9];         // viscous stress of the reference trackers
    R rho0, mu_s, lam_s;  // elasticity
    R c_light;            // Maxwell wave speed
    R cs2_phys;           // weakly compressible NSE: artificial sound speed squared
    R sq_ref;             // ultrarelativistic: sqrt(4 E0^2 - 3 |S0|^2)
    R inv_R_gas;          // 2D compressible NSF: 1 / R (T = p / (R rho))
    R inv_eta;            // homogenized NSF: drag rate 1 / eta
    R gen[16];            // generated systems: declared parameters, in order
    R H0[4];              // F0 - I (reference deformation minus identity)
    R P0[4];              // first Piola-Kirchhoff stress at F0
};

// d(a b / h) = ((a0 db + b0 da + da db) - dh a0 b0 / h0) / h for a = a0 + da,
// b = b0 + db, h = h0 + dh, with the reference ratio q0 = a0 b0 / h0 formed
// on the host: the deviation of a quotient of products without forming the
// products themselves.
template <class S, class R>
__host__ __device__ inline S dquot(R a0, R b0, R q0, const S &da, const S &db, const S &h, const S &dh)
{
    return ((a0 * db + b0 * da + da * db) - dh * q0) / h;
}

// ------------------------------------------------------------------ SWE --
// Shallow water (Sec. 3): Q = (h, hu, hv),
//   Phi_h = hu, Phi_hu = hu (x) u + g h^2/2 I, S_hu = -g h grad z_b.
struct SysSWE {
    static constexpr int K = 3, D = 2, id = 1;
    static constexpr bool precise = true;    // float-float equilibrium in single precision
    static constexpr bool compensated = true;   // two-sum moments dQ = hi + lo
    static constexpr bool tracker(int) { return false; }

    template <class S, class R>
    __host__ __device__ static void flux_delta(const Phys<R> &p, const S *dQ, S dPhi[][D])
    {
        const R h0 = p.Q0[0], mx0 = p.Q0[1], my0 = p.Q0[2];
        const S dh = dQ[0], dmx = dQ[1], dmy = dQ[2];
        const S h = dh + h0;
        const S pres = p.g * dh * (dh * R(0.5) + h0);          // g (h^2 - h0^2) / 2
        const S xy = dquot(mx0, my0, p.mm0_h0[1], dmx, dmy, h, dh);
        dPhi[0][0] = dmx;
        dPhi[0][1] = dmy;
        dPhi[1][0] = pres + dquot(mx0, mx0, p.mm0_h0[0], dmx, dmx, h, dh);
        dPhi[1][1] = xy;
        dPhi[2][0] = xy;
        dPhi[2][1] = pres + dquot(my0, my0, p.mm0_h0[2], dmy, dmy, h, dh);
    }

    template <class S, class R>
    __host__ __device__ static void source(const Phys<R> &p, const S *dQ, const R *b, S *Sk)
    {
        // b: the topography gradient of this cell (zeros when none is attached)
        const S h = dQ[0] + p.Q0[0];
        Sk[0] = S(R(0));
        Sk[1] = h * (-p.g * b[0]);
        Sk[2] = h * (-p.g * b[1]);
    }

    // largest |eigenvalue| of sum_a n_a A_a over unit n: |u| + sqrt(g h)
    template <class R>
    __host__ __device__ static R max_speed(const Phys<R> &p, const R *Q)
    {
        const R h = Q[0], ux = Q[1] / h, uy = Q[2] / h;
        return sqrt(ux * ux + uy * uy) + sqrt(p.g * h);
    }
};

// -------------------------------------------------------------- BURGERS --
// Inviscid Burgers (Sec. 3): Q = (u), Phi = (u^2 / 2, u^2 / 2), no source.
// d(u^2 / 2) = du (u0 + du / 2).
struct SysBurgers {
    static constexpr int K = 1, D = 2, id = 4;
    static constexpr bool precise = true;    // float-float equilibrium in single precision
    static constexpr bool compensated = true;   // two-sum moments dQ = hi + lo
    static constexpr bool tracker(int) { return false; }

    template <class S, class R>
    __host__ __device__ static void flux_delta(const Phys<R> &p, const S *dQ, S dPhi[][D])
    {
        const S du = dQ[0];
        const S d = du * (du * R(0.5) + p.Q0[0]);
        dPhi[0][0] = d;
        dPhi[0][1] = d;
    }

    template <class S, class R>
    __host__ __device__ static void source(const Phys<R> &, const S *, const R *, S *Sk)
    {
        Sk[0] = S(R(0));
    }

    // largest |eigenvalue| of sum_a n_a A_a over unit n: |u| |n0 + n1| <= sqrt(2) |u|
    template <class R>
    __host__ __device__ static R max_speed(const Phys<R> &, const R *Q)
    {
        return sqrt(R(2)) * fabs(Q[0]);
    }
};

// ---------------------------------------------------------------- EULER --
// Compressible Euler (Sec. 3): Q = (rho, m = rho u, E), ideal gas
// p = (gamma - 1)(E - |m|^2 / (2 rho)), Phi_rho = m, Phi_m = m (x) m / rho + p I,
// Phi_E = (E + p) m / rho, no source.  Fluctuation form: every quotient
// through dquot, dp = (gamma - 1)(dE - (d(mx mx/rho) + d(my my/rho)) / 2)
// and d(H m_c / rho) with H = E + p.
struct SysEuler {
    static constexpr int K = 4, D = 2, id = 5;
    static constexpr bool precise = true;    // float-float equilibrium in single precision
    static constexpr bool compensated = true;   // two-sum moments dQ = hi + lo
    static constexpr bool tracker(int) { return false; }

    template <class S, class R>
    __host__ __device__ static void flux_delta(const Phys<R> &p, const S *dQ, S dPhi[][D])
    {
        const R mx0 = p.Q0[1], my0 = p.Q0[2], H0 = p.H_ref;
        const S dr = dQ[0], dmx = dQ[1], dmy = dQ[2], dE = dQ[3];
        const S r = dr + p.Q0[0];
        const S xx = dquot(mx0, mx0, p.mm0_h0[0], dmx, dmx, r, dr);
        const S xy = dquot(mx0, my0, p.mm0_h0[1], dmx, dmy, r, dr);
        const S yy = dquot(my0, my0, p.mm0_h0[2], dmy, dmy, r, dr);
        const S dp = (p.gamma - R(1)) * (dE - (xx + yy) * R(0.5));
        const S dH = dE + dp;
        dPhi[0][0] = dmx;
        dPhi[0][1] = dmy;
        dPhi[1][0] = xx + dp;
        dPhi[1][1] = xy;
        dPhi[2][0] = xy;
        dPhi[2][1] = yy + dp;
        dPhi[3][0] = dquot(H0, mx0, p.Hu_ref[0], dH, dmx, r, dr);
        dPhi[3][1] = dquot(H0, my0, p.Hu_ref[1], dH, dmy, r, dr);
    }

    template <class S, class R>
    __host__ __device__ static void source(const Phys<R> &, const S *, const R *, S *Sk)
    {
#pragma unroll
        for (int k = 0; k < K; ++k) Sk[k] = S(R(0));
    }

    // |u| + c, c = sqrt(gamma p / rho)
    template <class R>
    __host__ __device__ static R max_speed(const Phys<R> &p, const R *Q)
    {
        const R r = Q[0], ux = Q[1] / r, uy = Q[2] / r;
        const R pr = (p.gamma - R(1)) * (Q[3] - R(0.5) * r * (ux * ux + uy * uy));
        return sqrt(ux * ux + uy * uy) + sqrt(p.gamma * (pr > R(0) ? pr : R(0)) / r);
    }
};

// -------------------------------------------------------------- MAXWELL --
// Maxwell, transverse-magnetic mode in vacuum (Sec. 3): Q = (E_z, H_x, H_y),
// Phi_Ez = c (-H_y, H_x), Phi_Hx = c (0, E_z), Phi_Hy = c (-E_z, 0), no
// source.  Linear, so dPhi is the flux of dQ.
struct SysMaxwell {
    static constexpr int K = 3, D = 2, id = 6;
    static constexpr bool precise = true;    // float-float equilibrium in single precision
    static constexpr bool compensated = true;   // two-sum moments dQ = hi + lo
    static constexpr bool tracker(int) { return false; }

    template <class S, class R>
    __host__ __device__ static void flux_delta(const Phys<R> &p, const S *dQ, S dPhi[][D])
    {
        const R c = p.c_light;
        dPhi[0][0] = dQ[2] * (-c);
        dPhi[0][1] = dQ[1] * c;
        dPhi[1][0] = S(R(0));
        dPhi[1][1] = dQ[0] * c;
        dPhi[2][0] = dQ[0] * (-c);
        dPhi[2][1] = S(R(0));
    }

    template <class S, class R>
    __host__ __device__ static void source(const Phys<R> &, const S *, const R *, S *Sk)
    {
#pragma unroll
        for (int k = 0; k < K; ++k) Sk[k] = S(R(0));
    }

    // flux Jacobian eigenvalues {+c, -c, 0} in every direction
    template <class R>
    __host__ __device__ static R max_speed(const Phys<R> &p, const R *)
    {
        return fabs(p.c_light);
    }
};

// ----------------------------------------------------------- ALLEN-CAHN --
// Allen-Cahn phase field with one gradient tracker (Sec. 3):
// Q = (phi, G), Phi_phi = -gamma G, Phi_G = -I phi / tau_grad,
// S_phi = r (phi - phi^3), S_G = -G / tau_grad; gamma in nu, r in react.
struct SysAllenCahn {
    static constexpr int K = 3, D = 2, id = 7;
    static constexpr bool precise = true;    // float-float equilibrium in single precision
    static constexpr bool compensated = true;   // two-sum moments dQ = hi + lo
    static constexpr bool tracker(int k) { return k > 0; }

    template <class S, class R>
    __host__ __device__ static void flux_delta(const Phys<R> &p, const S *dQ, S dPhi[][D])
    {
        const S dpi = dQ[0] * (-p.inv_tau_grad);
        dPhi[0][0] = dQ[1] * (-p.nu);
        dPhi[0][1] = dQ[2] * (-p.nu);
        dPhi[1][0] = dpi;
        dPhi[1][1] = S(R(0));
        dPhi[2][0] = S(R(0));
        dPhi[2][1] = dpi;
    }

    template <class S, class R>
    __host__ __device__ static void source(const Phys<R> &p, const S *dQ, const R *, S *Sk)
    {
        const S phi = dQ[0] + p.Q0[0];
        Sk[0] = (phi - phi * phi * phi) * p.react;
        Sk[1] = (dQ[1] + p.Q0[1]) * (-p.inv_tau_grad);
        Sk[2] = (dQ[2] + p.Q0[2]) * (-p.inv_tau_grad);
    }

    // eigenvalues of the (phi, G_n) block: +- sqrt(gamma / tau_grad)
    template <class R>
    __host__ __device__ static R max_speed(const Phys<R> &p, const R *)
    {
        return sqrt(p.nu * p.inv_tau_grad);
    }
};

// ------------------------------------------------------------ RELHYDRO --
// Ideal ultrarelativistic fluid, c = 1, p = e/3 (Sec. 3): Q = (E, S),
// p = (sqrt(4 E^2 - 3 |S|^2) - E) / 3, v = S / (E + p), Phi_E = S,
// Phi_S = S (x) v + p I = S (x) S / H + p I with H = E + p, no source.
// Fluctuation form: d sqrt = (4 dE (2 E0 + dE) - 3 dS.(2 S0 + dS)) /
// (sqrt + sqrt0), dp = (d sqrt - dE) / 3, S (x) S / H through dquot.
struct SysRelHydro {
    static constexpr int K = 3, D = 2, id = 8;
    static constexpr bool precise = true;    // float-float equilibrium in single precision
    static constexpr bool compensated = true;   // two-sum moments dQ = hi + lo
    static constexpr bool tracker(int) { return false; }

    template <class S, class R>
    __host__ __device__ static void flux_delta(const Phys<R> &p, const S *dQ, S dPhi[][D])
    {
        const R E0 = p.Q0[0], Sx0 = p.Q0[1], Sy0 = p.Q0[2];
        const S dE = dQ[0], dSx = dQ[1], dSy = dQ[2];
        const S E = dE + E0, Sx = dSx + Sx0, Sy = dSy + Sy0;
        const S sq = lbm_sqrt(E * E * R(4) - (Sx * Sx + Sy * Sy) * R(3));
        const S num = dE * (dE + R(2) * E0) * R(4) - (dSx * (dSx + R(2) * Sx0) + dSy * (dSy + R(2) * Sy0)) * R(3);
        const S dp = (num / (sq + p.sq_ref) - dE) * R(1.0 / 3.0);
        const S dH = dE + dp;
        const S H = dH + p.H_ref;
        const S xy = dquot(Sx0, Sy0, p.mm0_h0[1], dSx, dSy, H, dH);
        dPhi[0][0] = dSx;
        dPhi[0][1] = dSy;
        dPhi[1][0] = dquot(Sx0, Sx0, p.mm0_h0[0], dSx, dSx, H, dH) + dp;
        dPhi[1][1] = xy;
        dPhi[2][0] = xy;
        dPhi[2][1] = dquot(Sy0, Sy0, p.mm0_h0[2], dSy, dSy, H, dH) + dp;
    }

    template <class S, class R>
    __host__ __device__ static void source(const Phys<R> &, const S *, const R *, S *Sk)
    {
#pragma unroll
        for (int k = 0; k < K; ++k) Sk[k] = S(R(0));
    }

    // characteristic speeds of the massless gas never exceed c = 1
    template <class R>
    __host__ __device__ static R max_speed(const Phys<R> &, const R *)
    {
        return R(1);
    }
};

// ----------------------------------------------------------------- NSE --
// Weakly compressible Navier-Stokes with a momentum-gradient tracker
// (Sec. 3, incompressible limit): Q = (rho, m0, m1, G00, G01, G10, G11),
// G_ab ~ d_b m_a, Phi_m = m (x) m / rho + rho cs^2 I - mu (G + G^T) / rho,
// Phi_{G_ab, c} = G_ab m_c / rho - delta_bc m_a / tau_grad,
// S_G = -G / tau_grad.  Quotients through dquot; the reference ratios of
// the tracker rows are wave-uniform and formed in the kernel.
struct SysNSE {
    static constexpr int K = 7, D = 2, id = 9;
    static constexpr bool precise = true;    // float-float equilibrium in single precision
    static constexpr bool compensated = true;   // two-sum moments dQ = hi + lo
    static constexpr bool tracker(int k) { return k >= 3; }

    template <class S, class R>
    __host__ __device__ static void flux_delta(const Phys<R> &p, const S *dQ, S dPhi[][D])
    {
        const R r0 = p.Q0[0];
        const R m0[2] = {p.Q0[1], p.Q0[2]};
        const S dr = dQ[0];
        const S dm[2] = {dQ[1], dQ[2]};
        const S r = dr + r0;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            dPhi[0][c] = dm[c];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int q = a + c;                  // (0,0) -> 0, (0,1)/(1,0) -> 1, (1,1) -> 2
                const S conv = dquot(m0[a], m0[c], p.mm0_h0[q], dm[a], dm[c], r, dr);
                const R X0 = p.Q0[3 + 2 * a + c] + p.Q0[3 + 2 * c + a];
                const S dX = dQ[3 + 2 * a + c] + dQ[3 + 2 * c + a];
                const S visc = (dX - dr * (X0 / r0)) / r;
                dPhi[1 + a][c] = (a == c) ? conv + dr * p.cs2_phys - visc * p.mu : conv - visc * p.mu;
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const R G0 = p.Q0[3 + 2 * a + b];
                    const S tr = dquot(G0, m0[c], G0 * m0[c] / r0, dQ[3 + 2 * a + b], dm[c], r, dr);
                    dPhi[3 + 2 * a + b][c] = (b == c) ? tr - dm[a] * p.inv_tau_grad : tr;
                }
        }
    }

    template <class S, class R>
    __host__ __device__ static void source(const Phys<R> &p, const S *dQ, const R *, S *Sk)
    {
        Sk[0] = Sk[1] = Sk[2] = S(R(0));
#pragma unroll
        for (int k = 3; k < K; ++k) Sk[k] = (dQ[k] + p.Q0[k]) * (-p.inv_tau_grad);
    }

    // bound: |u| + cs + sqrt(2 mu / (rho tau_grad)) (acoustic plus the
    // tracker-coupled viscous modes)
    template <class R>
    __host__ __device__ static R max_speed(const Phys<R> &p, const R *Q)
    {
        const R ux = Q[1] / Q[0], uy = Q[2] / Q[0];
        return sqrt(ux * ux + uy * uy) + sqrt(p.cs2_phys) + sqrt(R(2) * p.mu * p.inv_tau_grad / Q[0]);
    }
};

// ------------------------------------------------------------- CNSF 2D --
// 2D compressible Navier-Stokes-Fourier with conserved-field gradient
// trackers (Sec. 3): Q = (rho, m0, m1, E, Grho_0, Grho_1, Gm_00, Gm_01,
// Gm_10, Gm_11, GE_0, GE_1), Gx_b ~ d_b x.  Velocity and temperature
// gradients by the chain rule (grad u_ab = (Gm_ab - u_a Grho_b) / rho,
// grad T from grad p and Grho), tau = mu (grad u + grad u^T - 2/3 div u I),
// Phi_m = m (x) u + p I - tau, Phi_E = (E + p) u - tau . u - K grad T,
// tracker rows Gx (x) u - I x / tau_grad, S_G = -G / tau_grad.
// Fluctuation form as for the 3D cascade: du = (dm - drho u0) / rho,
// d(a u_c) = da u_c + a0 du_c; the viscous and heat terms, small where the
// trackers are small, as value minus reference value.
struct SysCNSF2D {
    static constexpr int K = 12, D = 2, id = 10;
    static constexpr bool precise = false;   // plain exact-moment equilibrium (VALU budget)
    static constexpr bool compensated = true;   // two-sum moments dQ = hi + lo
    static constexpr bool tracker(int k) { return k >= 4; }

    // viscous stress tau and temperature gradient of an absolute state
    template <class S, class R>
    __host__ __device__ static void diffusive(const Phys<R> &p, const S &rho, const S *u, const S &pr, const S *Q,
                                              S tau[2][2], S *gT)
    {
        S du[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) du[a][b] = (Q[6 + 2 * a + b] - u[a] * Q[4 + b]) / rho;
        const S div = du[0][0] + du[1][1];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                tau[a][b] = (a == b) ? (du[a][b] + du[b][a] - div * R(2.0 / 3.0)) * p.mu
                                     : (du[a][b] + du[b][a]) * p.mu;
        const S ku = (u[0] * u[0] + u[1] * u[1]) * R(0.5);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const S gp = (Q[10 + b] - (u[0] * Q[6 + b] + u[1] * Q[8 + b]) + ku * Q[4 + b]) * (p.gamma - R(1));
            gT[b] = (gp - pr * Q[4 + b] / rho) * p.inv_R_gas / rho;
        }
    }

    template <class S, class R>
    __host__ __device__ static void flux_delta(const Phys<R> &p, const S *dQ, S dPhi[][D])
    {
        const S drho = dQ[0];
        const S rho = drho + p.Q0[0];
        const S irho = R(1) / rho;
        S u[2], du[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            du[a] = (dQ[1 + a] - drho * p.u_ref[a]) * irho;
            u[a] = du[a] + p.u_ref[a];
        }
        const S dk = (rho * (du[0] * (du[0] + R(2) * p.u_ref[0]) + du[1] * (du[1] + R(2) * p.u_ref[1]))
                      + drho * (p.u_ref[0] * p.u_ref[0] + p.u_ref[1] * p.u_ref[1])) * R(0.5);
        const S dp = (dQ[3] - dk) * (p.gamma - R(1));
        const S pr = dp + p.p_ref;
        // absolute tracker values and the diffusive terms at Q and at Q0
        S Qa[K];
#pragma unroll
        for (int k = 0; k < K; ++k) Qa[k] = dQ[k] + p.Q0[k];
        S tau[2][2], gT[2];
        diffusive<S, R>(p, rho, u, pr, Qa, tau, gT);
        R tau0[2][2], gT0[2];
        const R u0[2] = {p.u_ref[0], p.u_ref[1]};
        diffusive<R, R>(p, p.Q0[0], u0, p.p_ref, p.Q0, tau0, gT0);
        const S dH = dQ[3] + dp;                          // d(E + p)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            dPhi[0][c] = dQ[1 + c];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                S v = dQ[1 + a] * u[c] + du[c] * p.Q0[1 + a] - (tau[a][c] - tau0[a][c]);
                if (a == c) v = v + dp;
                dPhi[1 + a][c] = v;
            }
            const S tu = (tau[c][0] - tau0[c][0]) * u[0] + (tau[c][1] - tau0[c][1]) * u[1]
                         + du[0] * tau0[c][0] + du[1] * tau0[c][1];
            dPhi[3][c] = dH * u[c] + du[c] * p.H_ref - tu - (gT[c] - gT0[c]) * p.kappa;
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int k = 4 + 2 * j + b;
                    S v = dQ[k] * u[c] + du[c] * p.Q0[k];
                    if (b == c) v = v - dQ[j] * p.inv_tau_grad;
                    dPhi[k][c] = v;
                }
        }
    }

    template <class S, class R>
    __host__ __device__ static void source(const Phys<R> &p, const S *dQ, const R *, S *Sk)
    {
#pragma unroll
        for (int k = 0; k < 4; ++k) Sk[k] = S(R(0));
#pragma unroll
        for (int k = 4; k < K; ++k) Sk[k] = (dQ[k] + p.Q0[k]) * (-p.inv_tau_grad);
    }

    // |u| + adiabatic sound speed of the conserved (Euler) subsystem
    template <class R>
    __host__ __device__ static R max_speed(const Phys<R> &p, const R *Q)
    {
        const R rho = Q[0], u0 = Q[1] / rho, u1 = Q[2] / rho;
        const R pr = (p.gamma - R(1)) * (Q[3] - R(0.5) * rho * (u0 * u0 + u1 * u1));
        const R c2 = p.gamma * pr / rho;
        return sqrt(u0 * u0 + u1 * u1) + sqrt(c2 > R(0) ? c2 : R(0));
    }
};

// ----------------------------------------------------------------- MHD --
// 2D resistive compressible MHD with Powell divergence cleaning and
// conserved-field gradient trackers (Sec. 3): Q = (rho, m0, m1, E, B0, B1,
// then the tracker pairs G_x,b ~ d_b x of x = rho, m0, m1, E, B0, B1),
// p_gas = (gamma - 1)(E - |m|^2 / 2 rho - |B|^2 / 2), p_tot = p_gas + |B|^2 / 2,
// T = p_gas / rho, Phi_m = m (x) u + p_tot I - B (x) B - tau,
// Phi_E = (E + p_tot) u - B (u . B) - tau . u - K grad T + eta j x B,
// Phi_B = B (x) u - u (x) B - eta G_B, Powell sources -div B (B, u . B, u)
// with div B = tr G_B, gamma, mu, K = kappa, eta = nu.  Fluctuation form as
// for the 2D compressible NSF; the dissipative and Lorentz-resistive terms
// (small where the trackers are small) as value minus reference value.
struct SysMHD {
    static constexpr int K = 18, D = 2, id = 11;
    static constexpr bool precise = false;   // plain exact-moment equilibrium (VALU budget)
    static constexpr bool compensated = true;   // two-sum moments dQ = hi + lo
    static constexpr bool tracker(int k) { return k >= 6; }

    // tau, grad T and eta j x B of an absolute state
    template <class S, class R>
    __host__ __device__ static void diffusive(const Phys<R> &p, const S &rho, const S *u, const S &pg, const S *Q,
                                              S tau[2][2], S *gT, S *jxB)
    {
        S du[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) du[a][b] = (Q[8 + 2 * a + b] - u[a] * Q[6 + b]) / rho;
        const S div = du[0][0] + du[1][1];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                tau[a][b] = (a == b) ? (du[a][b] + du[b][a] - div * R(2.0 / 3.0)) * p.mu
                                     : (du[a][b] + du[b][a]) * p.mu;
        const S ku = (u[0] * u[0] + u[1] * u[1]) * R(0.5);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const S gp = (Q[12 + b] - (u[0] * Q[8 + b] + u[1] * Q[10 + b]) + ku * Q[6 + b]
                          - (Q[4] * Q[14 + b] + Q[5] * Q[16 + b])) * (p.gamma - R(1));
            gT[b] = (gp - pg * Q[6 + b] / rho) / rho;
        }
        const S j = (Q[16] - Q[15]) * p.nu;             // eta (d0 B1 - d1 B0)
        jxB[0] = -j * Q[5];
        jxB[1] = j * Q[4];
    }

    template <class S, class R>
    __host__ __device__ static void flux_delta(const Phys<R> &p, const S *dQ, S dPhi[][D])
    {
        const S drho = dQ[0];
        const S rho = drho + p.Q0[0];
        const S irho = R(1) / rho;
        S u[2], du[2], B[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            du[a] = (dQ[1 + a] - drho * p.u_ref[a]) * irho;
            u[a] = du[a] + p.u_ref[a];
            B[a] = dQ[4 + a] + p.Q0[4 + a];
        }
        const S dk = (rho * (du[0] * (du[0] + R(2) * p.u_ref[0]) + du[1] * (du[1] + R(2) * p.u_ref[1]))
                      + drho * (p.u_ref[0] * p.u_ref[0] + p.u_ref[1] * p.u_ref[1])) * R(0.5);
        const S dmag = dQ[4] * (dQ[4] * R(0.5) + p.Q0[4]) + dQ[5] * (dQ[5] * R(0.5) + p.Q0[5]);
        const S dpg = (dQ[3] - dk - dmag) * (p.gamma - R(1));
        const S dpt = dpg + dmag;
        S Qa[K];
#pragma unroll
        for (int k = 0; k < K; ++k) Qa[k] = dQ[k] + p.Q0[k];
        S tau[2][2], gT[2], jxB[2];
        diffusive<S, R>(p, rho, u, dpg + p.p_ref, Qa, tau, gT, jxB);
        R tau0[2][2], gT0[2], jxB0[2];
        const R u0[2] = {p.u_ref[0], p.u_ref[1]};
        diffusive<R, R>(p, p.Q0[0], u0, p.p_ref, p.Q0, tau0, gT0, jxB0);
        const S dH = dQ[3] + dpt;                         // d(E + p_tot)
        const R w0 = u0[0] * p.Q0[4] + u0[1] * p.Q0[5];   // u0 . B0
        const S dw = du[0] * B[0] + du[1] * B[1] + u0[0] * dQ[4] + u0[1] * dQ[5];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            dPhi[0][c] = dQ[1 + c];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                S v = dQ[1 + a] * u[c] + du[c] * p.Q0[1 + a] - (dQ[4 + a] * B[c] + dQ[4 + c] * p.Q0[4 + a])
                      - (tau[a][c] - tau0[a][c]);
                if (a == c) v = v + dpt;
                dPhi[1 + a][c] = v;
            }
            const S tu = (tau[c][0] - tau0[c][0]) * u[0] + (tau[c][1] - tau0[c][1]) * u[1]
                         + du[0] * tau0[c][0] + du[1] * tau0[c][1];
            dPhi[3][c] = dH * u[c] + du[c] * p.H_ref - (dQ[4 + c] * (dw + w0) + dw * p.Q0[4 + c]) - tu
                         - (gT[c] - gT0[c]) * p.kappa + (jxB[c] - jxB0[c]);
#pragma unroll
            for (int a = 0; a < 2; ++a)
                dPhi[4 + a][c] = (dQ[4 + a] * u[c] + du[c] * p.Q0[4 + a]) - (du[a] * B[c] + dQ[4 + c] * u0[a])
                                 - dQ[14 + 2 * a + c] * p.nu;
#pragma unroll
            for (int f = 0; f < 6; ++f)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const int k = 6 + 2 * f + b;
                    S v = dQ[k] * u[c] + du[c] * p.Q0[k];
                    if (b == c) v = v - dQ[f] * p.inv_tau_grad;
                    dPhi[k][c] = v;
                }
        }
    }

    template <class S, class R>
    __host__ __device__ static void source(const Phys<R> &p, const S *dQ, const R *, S *Sk)
    {
        const S rho = dQ[0] + p.Q0[0];
        const S u0 = (dQ[1] + p.Q0[1]) / rho, u1 = (dQ[2] + p.Q0[2]) / rho;
        const S B0 = dQ[4] + p.Q0[4], B1 = dQ[5] + p.Q0[5];
        const S divB = (dQ[14] + p.Q0[14]) + (dQ[17] + p.Q0[17]);
        Sk[0] = S(R(0));
        Sk[1] = -divB * B0;
        Sk[2] = -divB * B1;
        Sk[3] = -divB * (u0 * B0 + u1 * B1);
        Sk[4] = -divB * u0;
        Sk[5] = -divB * u1;
#pragma unroll
        for (int k = 6; k < K; ++k) Sk[k] = (dQ[k] + p.Q0[k]) * (-p.inv_tau_grad);
    }

    // |u| + sqrt(c^2 + |B|^2 / rho), a bound of the fast magnetosonic speed
    template <class R>
    __host__ __device__ static R max_speed(const Phys<R> &p, const R *Q)
    {
        const R rho = Q[0], u0 = Q[1] / rho, u1 = Q[2] / rho, b2 = Q[4] * Q[4] + Q[5] * Q[5];
        const R pg = (p.gamma - R(1)) * (Q[3] - R(0.5) * rho * (u0 * u0 + u1 * u1) - R(0.5) * b2);
        const R c2 = p.gamma * (pg > R(0) ? pg : R(0)) / rho + b2 / rho;
        return sqrt(u0 * u0 + u1 * u1) + sqrt(c2);
    }
};

// -------------------------------------------------------------- ADVDIFF --
// Scalar advection-diffusion-reaction with one gradient tracker (Sec. 3):
// Q = (c, G), Phi_c = c a - nu G, Phi_G = G (x) a - I c / tau_grad,
// S_c = R c (1 - c), S_G = -G / tau_grad.  The flux is linear, so dPhi is
// the flux of dQ.
struct SysAdvDiff {
    static constexpr int K = 3, D = 2, id = 0;
    static constexpr bool precise = true;    // float-float equilibrium in single precision
    static constexpr bool compensated = true;   // two-sum moments dQ = hi + lo
    static constexpr bool tracker(int k) { return k > 0; }

    template <class S, class R>
    __host__ __device__ static void flux_delta(const Phys<R> &p, const S *dQ, S dPhi[][D])
    {
        const S dc = dQ[0];
        const S dci = dc * p.inv_tau_grad;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            dPhi[0][a] = dc * p.a[a] - dQ[1 + a] * p.nu;
#pragma unroll
            for (int b = 0; b < D; ++b)
                dPhi[1 + b][a] = (a == b) ? dQ[1 + b] * p.a[a] - dci : dQ[1 + b] * p.a[a];
        }
    }

    template <class S, class R>
    __host__ __device__ static void source(const Phys<R> &p, const S *dQ, const R *, S *Sk)
    {
        const S c = dQ[0] + p.Q0[0];
        Sk[0] = c * (R(1) - c) * p.react;
        Sk[1] = (dQ[1] + p.Q0[1]) * (-p.inv_tau_grad);
        Sk[2] = (dQ[2] + p.Q0[2]) * (-p.inv_tau_grad);
    }

    // eigenvalues of the (c, G_n) block: a.n +- sqrt(nu / tau_grad)
    template <class R>
    __host__ __device__ static R max_speed(const Phys<R> &p, const R *)
    {
        return sqrt(p.a[0] * p.a[0] + p.a[1] * p.a[1]) + sqrt(p.nu * p.inv_tau_grad);
    }
};

// ------------------------------------------------------------- NEOHOOKE --
// Neo-Hookean elasticity, total-Lagrangian, momentum divided by rho0
// (Sec. 3): Q = (F00, F01, F10, F11, v0, v1),
//   Phi_{F_ab, c} = -v_a delta_bc,  Phi_{v_a, c} = -P_ac / rho0,
//   P = mu_s (F - F^{-T}) + lambda_s ln J F^{-T},  S = 0.
// With H = F - I: J - 1 = H00 + H11 + H00 H11 - H01 H10, cof F = J F^{-T},
// F - F^{-T} = (J F - cof F) / J, all formed from the small entries of H.
struct SysNeoHooke {
    static constexpr int K = 6, D = 2, id = 2;
    static constexpr bool precise = true;    // float-float equilibrium in single precision
    static constexpr bool compensated = true;   // two-sum moments dQ = hi + lo
    static constexpr bool tracker(int) { return false; }

    template <class S, class R>
    __host__ __device__ static void stress(const Phys<R> &p, const S H[4], S P[4])
    {
        const S dJ = H[0] + H[3] + H[0] * H[3] - H[1] * H[2];
        const S invJ = R(1) / (dJ + R(1));
        const S lnJ = lbm_log1p(dJ);
        // cof F = [[1 + H11, -H10], [-H01, 1 + H00]]
        const S c00 = H[3] + R(1), c01 = -H[2], c10 = -H[1], c11 = H[0] + R(1);
        // J F - cof F
        const S e00 = dJ + H[0] + dJ * H[0] - H[3];
        const S e01 = H[1] + H[2] + dJ * H[1];
        const S e10 = H[2] + H[1] + dJ * H[2];
        const S e11 = dJ + H[3] + dJ * H[3] - H[0];
        P[0] = (e00 * p.mu_s + lnJ * c00 * p.lam_s) * invJ;
        P[1] = (e01 * p.mu_s + lnJ * c01 * p.lam_s) * invJ;
        P[2] = (e10 * p.mu_s + lnJ * c10 * p.lam_s) * invJ;
        P[3] = (e11 * p.mu_s + lnJ * c11 * p.lam_s) * invJ;
    }

    template <class S, class R>
    __host__ __device__ static void flux_delta(const Phys<R> &p, const S *dQ, S dPhi[][D])
    {
        S H[4], P[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) H[j] = dQ[j] + p.H0[j];
        stress(p, H, P);
        const R ir = R(1) / p.rho0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c) dPhi[2 * a + b][c] = (b == c) ? -dQ[4 + a] : S(R(0));
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < 2; ++c) dPhi[4 + a][c] = (P[2 * a + c] - p.P0[2 * a + c]) * (-ir);
    }

    template <class S, class R>
    __host__ __device__ static void source(const Phys<R> &, const S *, const R *, S *Sk)
    {
#pragma unroll
        for (int k = 0; k < K; ++k) Sk[k] = S(R(0));
    }

    // largest elastic wave speed: sqrt of the largest eigenvalue of the
    // acoustic tensor A_ac(n) = (1/rho0) dP_ab/dF_cd n_b n_d over 16 directions
    template <class R>
    __host__ __device__ static R max_speed(const Phys<R> &p, const R *Q)
    {
        using DD = Dual<R, 4>;
        DD H[4], P[4];
        for (int j = 0; j < 4; ++j) {
            H[j] = DD(Q[j] - (j == 0 || j == 3 ? R(1) : R(0)));
            H[j].d[j] = R(1);
        }
        stress(p, H, P);
        R best = R(0);
        for (int s = 0; s < 16; ++s) {
            const R th = R(3.14159265358979323846) * R(s) / R(16);
            const R n[2] = {cos(th), sin(th)};
            R A[2][2];
            for (int a = 0; a < 2; ++a)
                for (int c = 0; c < 2; ++c) {
                    R acc = R(0);
                    for (int b = 0; b < 2; ++b)
                        for (int d = 0; d < 2; ++d) acc += P[2 * a + b].d[2 * c + d] * n[b] * n[d];
                    A[a][c] = acc / p.rho0;
                }
            const R tr = A[0][0] + A[1][1];
            const R det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
            const R disc = tr * tr * R(0.25) - det;
            const R lmax = tr * R(0.5) + sqrt(disc > R(0) ? disc : R(0));
            const R c = sqrt(lmax > R(0) ? lmax : R(0));
            best = c > best ? c : best;
        }
        return best;
    }
};

// ---------------------------------------------------------------- NSF17 --
// 3D compressible Navier-Stokes-Fourier with derived-field gradient
// trackers (Sec. 3, compressible NSF; homogenized NSF at porosity 1 with the
// full velocity-gradient basis; tracker construction of Sec. 2.1.1):
//   Q = (rho, m, E, G_ab ~ d_b u_a, G_T ~ grad T), u = m/rho,
//   p = (gamma-1)(E - |m|^2/(2 rho)), T = p/rho,
//   tau = mu (G + G^T - 2/3 tr G I),
//   Phi_rho = m, Phi_m = m (x) u + p I - tau,
//   Phi_E = (E + p) u - tau u - kappa G_T,
//   Phi_{G_ab, c} = G_ab u_c - delta_bc u_a / tau_grad,
//   Phi_{G_Ta, c} = G_Ta u_c - delta_ac T / tau_grad,
//   S_G = -G / tau_grad (zero for the conserved rows).
// Fluctuation form: du = (dm - drho u0)/rho, dp = (gamma-1)(dE - dk) with
// dk = (rho du.(2 u0 + du) + drho |u0|^2)/2, dT = (dp - T0 drho)/rho, and
// every product ab - a0 b0 written as da b + a0 db.
struct SysNSF17 {
    static constexpr int K = 17, D = 3, id = 3;
    static constexpr bool precise = false;   // no dual-number flux correction (register budget)
    static constexpr bool ffeq = true;       // float-float equilibria from the plain-float flux
    static constexpr bool compensated = true;   // two-sum moments dQ = hi + lo
    static constexpr bool tracker(int k) { return k >= 5; }

    template <class S, class R>
    __host__ __device__ static void flux_delta(const Phys<R> &p, const S *dQ, S dPhi[][D])
    {
        const S drho = dQ[0];
        const S rho = drho + p.Q0[0];
        const S irho = R(1) / rho;
        S u[3], du[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            du[a] = (dQ[1 + a] - drho * p.u_ref[a]) * irho;
            u[a] = du[a] + p.u_ref[a];
        }
        const S dk = (rho * (du[0] * (du[0] + R(2) * p.u_ref[0]) + du[1] * (du[1] + R(2) * p.u_ref[1])
                             + du[2] * (du[2] + R(2) * p.u_ref[2]))
                      + drho * (p.u_ref[0] * p.u_ref[0] + p.u_ref[1] * p.u_ref[1] + p.u_ref[2] * p.u_ref[2]))
                     * R(0.5);
        const S dp = (dQ[4] - dk) * (p.gamma - R(1));
        const S dT = (dp - drho * p.T_ref) * irho;
        // deviation of the viscous stress (linear in the trackers)
        const S trG = dQ[5] + dQ[9] + dQ[13];
        S dtau[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                dtau[a][b] = (dQ[5 + 3 * a + b] + dQ[5 + 3 * b + a] - (a == b ? trG * R(2.0 / 3.0) : S(R(0)))) * p.mu;
        const S dH = dQ[4] + dp;                          // d(E + p)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dPhi[0][c] = dQ[1 + c];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                S v = dQ[1 + a] * u[c] + du[c] * p.Q0[1 + a] - dtau[a][c];
                if (a == c) v = v + dp;
                dPhi[1 + a][c] = v;
            }
            S tu = dtau[c][0] * u[0] + dtau[c][1] * u[1] + dtau[c][2] * u[2]
                   + du[0] * p.tau_ref[3 * c + 0] + du[1] * p.tau_ref[3 * c + 1] + du[2] * p.tau_ref[3 * c + 2];
            dPhi[4][c] = dH * u[c] + du[c] * p.H_ref - tu - dQ[14 + c] * p.kappa;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    S v = dQ[5 + 3 * a + b] * u[c] + du[c] * p.Q0[5 + 3 * a + b];
                    if (b == c) v = v - du[a] * p.inv_tau_grad;
                    dPhi[5 + 3 * a + b][c] = v;
                }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                S v = dQ[14 + a] * u[c] + du[c] * p.Q0[14 + a];
                if (a == c) v = v - dT * p.inv_tau_grad;
                dPhi[14 + a][c] = v;
            }
        }
    }

    template <class S, class R>
    __host__ __device__ static void source(const Phys<R> &p, const S *dQ, const R *, S *Sk)
    {
#pragma unroll
        for (int k = 0; k < 5; ++k) Sk[k] = S(R(0));
#pragma unroll
        for (int k = 5; k < K; ++k) Sk[k] = (dQ[k] + p.Q0[k]) * (-p.inv_tau_grad);
    }

    // |u| + adiabatic sound speed of the conserved (Euler) subsystem
    template <class R>
    __host__ __device__ static R max_speed(const Phys<R> &p, const R *Q)
    {
        const R rho = Q[0];
        const R u0 = Q[1] / rho, u1 = Q[2] / rho, u2 = Q[3] / rho;
        const R pr = (p.gamma - R(1)) * (Q[4] - R(0.5) * rho * (u0 * u0 + u1 * u1 + u2 * u2));
        const R c2 = p.gamma * pr / rho;
        return sqrt(u0 * u0 + u1 * u1 + u2 * u2) + sqrt(c2 > R(0) ? c2 : R(0));
    }
};

// ---------------------------------------------------------------- HCNSF --
// Homogenized compressible NSF in 3D (Sec. 3, homogenized NSF) with the
// strain-reduced tracker basis: Q = (rho, rho u, E, G_u, G_T) with
// G_u = sym grad u stored as (00, 11, 22, 01, 02, 12) and G_T = grad T,
// T = p / rho, 14 fields.  Prescribed per-cell coefficients (alpha, u_s):
// porosity alpha scales the viscous stress and the heat flux, and the drag
// (1 - alpha) / eta (rho u_s - rho u) forces momentum and energy.
//   Phi_m  = m u^T + p I - alpha tau,  tau = mu (2 G_u - 2/3 tr(G_u) I)
//   Phi_E  = (E + p) u - alpha tau u - alpha kappa G_T
//   Phi_Gu = G_u u^T - sym(I (x) u) / tau_grad,  Phi_GT = G_T u^T - T I / tau_grad
// The reference trackers are zero (the library enforces it), so the
// reference flux does not depend on alpha and the deviation of the
// dissipative terms is the terms themselves.
struct SysHCNSF {
    static constexpr int K = 14, D = 3, id = 12;
    static constexpr bool precise = false;   // no dual-number flux correction (register budget)
    static constexpr bool ffeq = true;       // float-float equilibria from the plain-float flux
    static constexpr bool compensated = true;
    static constexpr bool tracker(int k) { return k >= 5; }
    // coefficient field: 4 values per cell, read by the flux as well
    static constexpr int NB = 4;
    static constexpr bool coef_in_flux = true;
    __host__ __device__ static constexpr double coef_default(int a) { return a == 0 ? 1.0 : 0.0; }

    template <class S, class R>
    __host__ __device__ static void flux_delta_b(const Phys<R> &p, const S *dQ, const R *b, S dPhi[][D])
    {
        const S drho = dQ[0];
        const S rho = drho + p.Q0[0];
        const S irho = R(1) / rho;
        S u[3], du[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            du[a] = (dQ[1 + a] - drho * p.u_ref[a]) * irho;
            u[a] = du[a] + p.u_ref[a];
        }
        const S dk = (rho * (du[0] * (du[0] + R(2) * p.u_ref[0]) + du[1] * (du[1] + R(2) * p.u_ref[1])
                             + du[2] * (du[2] + R(2) * p.u_ref[2]))
                      + drho * (p.u_ref[0] * p.u_ref[0] + p.u_ref[1] * p.u_ref[1] + p.u_ref[2] * p.u_ref[2]))
                     * R(0.5);
        const S dp = (dQ[4] - dk) * (p.gamma - R(1));
        const S dT = (dp - drho * p.T_ref) * irho;
        // alpha tau from the strain trackers (symmetric)
        const R amu = b[0] * p.mu, akappa = b[0] * p.kappa;
        const S tr3 = (dQ[5] + dQ[6] + dQ[7]) * R(2.0 / 3.0);
        S at[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) at[a][a] = (R(2) * dQ[5 + a] - tr3) * amu;
        at[0][1] = at[1][0] = R(2) * dQ[8] * amu;
        at[0][2] = at[2][0] = R(2) * dQ[9] * amu;
        at[1][2] = at[2][1] = R(2) * dQ[10] * amu;
        const S dH = dQ[4] + dp;                          // d(E + p)
        const R half_itg = R(0.5) * p.inv_tau_grad;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            dPhi[0][c] = dQ[1 + c];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                S v = dQ[1 + a] * u[c] + du[c] * p.Q0[1 + a] - at[a][c];
                if (a == c) v = v + dp;
                dPhi[1 + a][c] = v;
            }
            dPhi[4][c] = dH * u[c] + du[c] * p.H_ref - (at[c][0] * u[0] + at[c][1] * u[1] + at[c][2] * u[2])
                         - dQ[11 + c] * akappa;
            // diagonal strain trackers: - delta_ac du_a / tau_grad
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                S v = dQ[5 + a] * u[c];
                if (a == c) v = v - du[a] * p.inv_tau_grad;
                dPhi[5 + a][c] = v;
            }
            // off-diagonal (01, 02, 12): - (delta_bc du_a + delta_ac du_b) / (2 tau_grad)
            {
                S v01 = dQ[8] * u[c], v02 = dQ[9] * u[c], v12 = dQ[10] * u[c];
                if (c == 0) { v01 = v01 - du[1] * half_itg; v02 = v02 - du[2] * half_itg; }
                if (c == 1) { v01 = v01 - du[0] * half_itg; v12 = v12 - du[2] * half_itg; }
                if (c == 2) { v02 = v02 - du[0] * half_itg; v12 = v12 - du[1] * half_itg; }
                dPhi[8][c] = v01;
                dPhi[9][c] = v02;
                dPhi[10][c] = v12;
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                S v = dQ[11 + a] * u[c];
                if (a == c) v = v - dT * p.inv_tau_grad;
                dPhi[11 + a][c] = v;
            }
        }
    }

    template <class S, class R>
    __host__ __device__ static void source(const Phys<R> &p, const S *dQ, const R *b, S *Sk)
    {
        const S rho = dQ[0] + p.Q0[0];
        const R drag = (R(1) - b[0]) * p.inv_eta;
        Sk[0] = S(R(0));
        S se = S(R(0));
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const S m = dQ[1 + a] + p.Q0[1 + a];
            const S sm = (rho * b[1 + a] - m) * drag;
            Sk[1 + a] = sm;
            se = se + sm * (m / rho);
        }
        Sk[4] = se;
#pragma unroll
        for (int k = 5; k < K; ++k) Sk[k] = (dQ[k] + p.Q0[k]) * (-p.inv_tau_grad);
    }

    template <class R>
    __host__ __device__ static R max_speed(const Phys<R> &p, const R *Q)
    {
        return SysNSF17::max_speed(p, Q);
    }
};

// Per-cell coefficient field of a system: NB values per cell ([NB][cells]),
// read by the source and, where coef_in_flux, by the flux; missing values
// take coef_default.  Systems without these members read D values (the
// topography gradient of SWE), zero when no field is attached.
template <class S, class = void>
struct CoefTraits {
    static constexpr int NB = S::D;
    static constexpr bool in_flux = false;
    __host__ __device__ static constexpr double dflt(int) { return 0.0; }
};
template <class S>
struct CoefTraits<S, std::void_t<decltype(S::NB)>> {
    static constexpr int NB = S::NB;
    static constexpr bool in_flux = S::coef_in_flux;
    __host__ __device__ static constexpr double dflt(int a) { return S::coef_default(a); }
};
