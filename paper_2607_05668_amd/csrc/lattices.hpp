// Velocity sets of the collide-and-stream library (compile-time tables).
//
// Each lattice satisfies the isotropy conditions of Sec. 2.2: the weights
// sum to one, their first moment vanishes and their second moment is
// cs^2 times the identity.  D2Q5 and D3Q7 follow the supplement's stencil
// table; D2Q9 uses the standard 4/9, 1/9, 1/36 weights.  The population
// order is part of the ABI (see include/lbm.h).
#pragma once

struct D2Q5 {
    static constexpr int D = 2, Q = 5;
    static constexpr int cx[Q] = {0, 1, 0, -1, 0};
    static constexpr int cy[Q] = {0, 0, 1, 0, -1};
    static constexpr int cz[Q] = {0, 0, 0, 0, 0};
    static constexpr double w[Q] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
    static constexpr double cs2 = 1.0 / 3;
    static constexpr int id = 0;
    // w_i = Wn_i / Wden;  w_i / cs^2 = Wn_i / Fden
    static constexpr int Wn[Q] = {2, 1, 1, 1, 1};
    static constexpr int Wden = 6, Fden = 2;
};

struct D2Q9 {
    static constexpr int D = 2, Q = 9;
    static constexpr int cx[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int cy[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int cz[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    static constexpr double w[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    static constexpr double cs2 = 1.0 / 3;
    static constexpr int id = 1;
    static constexpr int Wn[Q] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
    static constexpr int Wden = 36, Fden = 12;
};

struct D3Q7 {
    static constexpr int D = 3, Q = 7;
    static constexpr int cx[Q] = {0, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[Q] = {0, 0, 0, 1, -1, 0, 0};
    static constexpr int cz[Q] = {0, 0, 0, 0, 0, 1, -1};
    static constexpr double w[Q] = {1.0 / 4, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8};
    static constexpr double cs2 = 1.0 / 4;
    static constexpr int id = 2;
    static constexpr int Wn[Q] = {2, 1, 1, 1, 1, 1, 1};
    static constexpr int Wden = 8, Fden = 2;
};

// c_{i,a} as a compile-time function of (i, a)
template <class L>
__host__ __device__ constexpr int lat_c(int i, int a)
{
    return a == 0 ? L::cx[i] : (a == 1 ? L::cy[i] : L::cz[i]);
}

// Exact-moment equilibrium.  With e_i = w_i dQ + (w_i / cs^2) c_i . G,
// G = (dt/dx) dPhi, the weights are written as exact rationals so that in
// floating point the lattice moments of e carry only value-dependent
// (unbiased) rounding: w_i dQ is one correctly rounded division followed by
// power-of-two scalings, and the flux part is G / 3 (D2Q9) or G / 2 (D2Q5,
// D3Q7) with power-of-two scalings.  Rounding the weights themselves would
// bias every cell's moments by the same relative amount, which the nearly
// undamped non-equilibrium moments at omega -> 2 accumulate.  e_0 (rest) is
// not formed: the collision closes the zeroth moment through the rest
// population.  The zeroth part takes the moment as an unevaluated sum
// dQ = hi + lo (compensated summation), w_i dQ = w_i hi + w_i lo.
// `zeroth` gives w_i s for i >= 1 (used for the source term).
template <class L> struct ExactEq;

template <> struct ExactEq<D2Q5> {
    template <class R> __host__ __device__ static void feq(R hi, R lo, const R *G, R *e)
    {
        const R A = hi / R(6) + lo / R(6), hx = G[0] * R(0.5), hy = G[1] * R(0.5);
        e[1] = A + hx; e[2] = A + hy; e[3] = A - hx; e[4] = A - hy;
    }
    template <class R> __host__ __device__ static void zeroth(R s, R *e)
    {
        const R A = s / R(6);
        e[1] = A; e[2] = A; e[3] = A; e[4] = A;
    }
};

template <> struct ExactEq<D2Q9> {
    template <class R> __host__ __device__ static void feq(R hi, R lo, const R *G, R *e)
    {
        const R A = hi / R(36) + lo / R(36), A4 = A * R(4);
        const R gx = G[0] / R(3), gy = G[1] / R(3);
        e[1] = A4 + gx; e[2] = A4 + gy; e[3] = A4 - gx; e[4] = A4 - gy;
        e[5] = A + (gx + gy) * R(0.25); e[6] = A + (gy - gx) * R(0.25);
        e[7] = A - (gx + gy) * R(0.25); e[8] = A + (gx - gy) * R(0.25);
    }
    template <class R> __host__ __device__ static void zeroth(R s, R *e)
    {
        const R A = s / R(36), A4 = A * R(4);
        e[1] = A4; e[2] = A4; e[3] = A4; e[4] = A4;
        e[5] = A; e[6] = A; e[7] = A; e[8] = A;
    }
};

template <> struct ExactEq<D3Q7> {
    template <class R> __host__ __device__ static void feq(R hi, R lo, const R *G, R *e)
    {
        const R A = hi * R(0.125) + lo * R(0.125), hx = G[0] * R(0.5), hy = G[1] * R(0.5), hz = G[2] * R(0.5);
        e[1] = A + hx; e[2] = A - hx; e[3] = A + hy; e[4] = A - hy; e[5] = A + hz; e[6] = A - hz;
    }
    template <class R> __host__ __device__ static void zeroth(R s, R *e)
    {
        const R A = s * R(0.125);
        for (int i = 1; i < 7; ++i) e[i] = A;
    }
};
