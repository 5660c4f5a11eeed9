// Velocity sets of the collide-and-stream library (compile-time tables).
//
// Each lattice satisfies the isotropy conditions of Sec. 2.2: the weights
// sum to one, their first moment vanishes and their second moment is
// cs^2 times the identity.  D2Q5 and D3Q7 follow the supplement's stencil
// table; D2Q9 uses the standard 4/9, 1/9, 1/36 weights.  The population
// order is part of the ABI (see include/lbm.h).
#pragma once

#include <type_traits>

// x / D, correctly rounded, for the weight denominators D = 3 and 9 in
// single precision without a division instruction: q0 = x RN(1/D) is within
// an ulp of x / D, the remainder x - q0 D is exact (fma), and one correction
// q0 + r RN(1/D) rounds to the quotient.  For these two divisors the result
// equals the IEEE quotient for every finite float (checked exhaustively over
// all 2^31 magnitudes, subnormals included); 6 and 36 are reached through
// power-of-two scalings, exact wherever the quotient is a normal number.
// Other precisions divide.
template <int D, class R>
__host__ __device__ inline R div_by(R x)
{
    if constexpr (std::is_same<R, float>::value && (D == 3 || D == 9)) {
        constexpr float r = 1.0f / D;
        const float q0 = x * r;
        return fmaf(fmaf(-q0, (float)D, x), r, q0);
    } else {
        return x / R(D);
    }
}

struct D2Q5 {
    static constexpr int D = 2, Q = 5;
    static constexpr int cx[Q] = {0, 1, 0, -1, 0};
    static constexpr int cy[Q] = {0, 0, 1, 0, -1};
    static constexpr int cz[Q] = {0, 0, 0, 0, 0};
    static constexpr int opp[Q] = {0, 3, 4, 1, 2};       // index of -c_i
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
    static constexpr int opp[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
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
    static constexpr int opp[Q] = {0, 2, 1, 4, 3, 6, 5};
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
// (unbiased) rounding: w_i dQ is one correctly rounded division (div_by)
// followed by power-of-two scalings, and the flux part is G / 3 (D2Q9) or G / 2 (D2Q5,
// D3Q7) with power-of-two scalings.  Rounding the weights themselves would
// bias every cell's moments by the same relative amount, which the nearly
// undamped non-equilibrium moments at omega -> 2 accumulate.  e_0 (rest) is
// not formed: the collision closes the zeroth moment through the rest
// population (`rest` gives w_0 M in the same exact form where a rest value is
// needed).  The zeroth part takes the moment as an unevaluated sum
// dQ = hi + lo (compensated summation), w_i dQ = w_i hi + w_i lo.
// `zeroth` gives w_i s for i >= 1 (used for the source term).
template <class L> struct ExactEq;

template <> struct ExactEq<D2Q5> {
    template <class R> __host__ __device__ static R rest(R M) { return div_by<3>(M); }
    template <class R> __host__ __device__ static R amp(R qh, R ql) { return qh * R(0.5) + ql * R(0.5); }
    template <class R> __host__ __device__ static R comb(R A, R hx, R hy, int i)
    {
        return i == 1 ? A + hx : (i == 2 ? A + hy : (i == 3 ? A - hx : A - hy));
    }
    template <class R> __host__ __device__ static void feq(R hi, R lo, const R *G, R *e)
    {
        const R A = amp(div_by<3>(hi), div_by<3>(lo)), hx = G[0] * R(0.5), hy = G[1] * R(0.5);
#pragma unroll
        for (int i = 1; i < 5; ++i) e[i] = comb(A, hx, hy, i);
    }
    // One sender's equilibrium rebuilt direction by direction (lo = 0):
    // parts() forms its per-cell quantities once, rest_parts() and dir()
    // finish w_0 M and e_i with the operations of rest() and feq(), so
    // dir(parts(M, G), i) equals feq(M, 0, G)[i] bit for bit.
    template <class R> __host__ __device__ static void parts(R M, const R *G, R *P)
    {
        P[0] = div_by<3>(M); P[1] = G[0] * R(0.5); P[2] = G[1] * R(0.5);
    }
    template <class R> __host__ __device__ static R rest_parts(const R *P) { return P[0]; }
    template <class R> __host__ __device__ static R dir(const R *P, int i)
    {
        return comb(amp(P[0], div_by<3>(R(0))), P[1], P[2], i);
    }
    template <class R> __host__ __device__ static void zeroth(R s, R *e)
    {
        const R A = div_by<3>(s) * R(0.5);
        e[1] = A; e[2] = A; e[3] = A; e[4] = A;
    }
};

template <> struct ExactEq<D2Q9> {
    template <class R> __host__ __device__ static R rest(R M) { return div_by<9>(M) * R(4); }
    template <class R> __host__ __device__ static R amp(R qh, R ql) { return qh * R(0.25) + ql * R(0.25); }
    template <class R> __host__ __device__ static R comb(R A, R gx, R gy, int i)
    {
        const R A4 = A * R(4);
        switch (i) {
        case 1: return A4 + gx;
        case 2: return A4 + gy;
        case 3: return A4 - gx;
        case 4: return A4 - gy;
        case 5: return A + (gx + gy) * R(0.25);
        case 6: return A + (gy - gx) * R(0.25);
        case 7: return A - (gx + gy) * R(0.25);
        default: return A + (gx - gy) * R(0.25);
        }
    }
    template <class R> __host__ __device__ static void feq(R hi, R lo, const R *G, R *e)
    {
        const R A = amp(div_by<9>(hi), div_by<9>(lo));
        const R gx = div_by<3>(G[0]), gy = div_by<3>(G[1]);
#pragma unroll
        for (int i = 1; i < 9; ++i) e[i] = comb(A, gx, gy, i);
    }
    // per-sender parts and the direction-wise rebuild, as for D2Q5
    template <class R> __host__ __device__ static void parts(R M, const R *G, R *P)
    {
        P[0] = div_by<9>(M); P[1] = div_by<3>(G[0]); P[2] = div_by<3>(G[1]);
    }
    template <class R> __host__ __device__ static R rest_parts(const R *P) { return P[0] * R(4); }
    template <class R> __host__ __device__ static R dir(const R *P, int i)
    {
        return comb(amp(P[0], div_by<9>(R(0))), P[1], P[2], i);
    }
    template <class R> __host__ __device__ static void zeroth(R s, R *e)
    {
        const R A = div_by<9>(s) * R(0.25), A4 = A * R(4);
        e[1] = A4; e[2] = A4; e[3] = A4; e[4] = A4;
        e[5] = A; e[6] = A; e[7] = A; e[8] = A;
    }
};

template <> struct ExactEq<D3Q7> {
    template <class R> __host__ __device__ static R rest(R M) { return M * R(0.25); }
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

// Float-float form of the same equilibrium, for single-precision arithmetic:
// every quantity is an unevaluated pair (hi, lo) built with error-free
// transformations (two-sum; exact division remainder r = a - q b and exact
// product error via fused multiply-add), so that e_i carries no rounding
// beyond ~2^-44 relative and the collision rounds only once, at the store.
template <class R>
struct FF {
    R hi, lo;
};

template <class R>
__host__ __device__ inline FF<R> ff_two_sum(R a, R b)
{
    const R s = a + b;
    const R bp = s - a;
    return {s, (a - (s - bp)) + (b - bp)};
}

template <class R>
__host__ __device__ inline FF<R> ff_add(FF<R> a, FF<R> b)
{
    FF<R> s = ff_two_sum(a.hi, b.hi);
    s.lo += a.lo + b.lo;
    return s;
}

// (hi + lo) / (B P) for B = 3 or 9 and a power of two P: q = RN(hi / (B P)),
// the remainder hi - q B P is exact, and the low part (r + lo) / (B P) needs
// no correct rounding (a product with the rounded reciprocal).
template <int B, class R>
__host__ __device__ inline FF<R> ff_div(R hi, R lo, R P)
{
    const R q = div_by<B>(hi) / P;
    const R r = fma(-q, R(B) * P, hi);
    return {q, (r + lo) * (R(1) / (R(B) * P))};
}

template <class R>
__host__ __device__ inline FF<R> ff_scale(FF<R> a, R s)      // s a power of two
{
    return {a.hi * s, a.lo * s};
}

// e_i (i >= 1) as float-float pairs from dQ = (qh, ql) and G = (Gh, Gl)
template <class L> struct ExactEqFF;

template <> struct ExactEqFF<D2Q5> {
    template <class R>
    __host__ __device__ static void feq(R qh, R ql, const R *Gh, const R *Gl, FF<R> *e)
    {
        const FF<R> A = ff_div<3>(qh, ql, R(2));
        const FF<R> hx = {Gh[0] * R(0.5), Gl[0] * R(0.5)}, hy = {Gh[1] * R(0.5), Gl[1] * R(0.5)};
        const FF<R> mhx = {-hx.hi, -hx.lo}, mhy = {-hy.hi, -hy.lo};
        e[1] = ff_add(A, hx); e[2] = ff_add(A, hy); e[3] = ff_add(A, mhx); e[4] = ff_add(A, mhy);
    }
};

template <> struct ExactEqFF<D2Q9> {
    template <class R>
    __host__ __device__ static void feq(R qh, R ql, const R *Gh, const R *Gl, FF<R> *e)
    {
        const FF<R> A = ff_div<9>(qh, ql, R(4)), A4 = ff_scale(A, R(4));
        const FF<R> gx = ff_div<3>(Gh[0], Gl[0], R(1)), gy = ff_div<3>(Gh[1], Gl[1], R(1));
        const FF<R> mgx = {-gx.hi, -gx.lo}, mgy = {-gy.hi, -gy.lo};
        e[1] = ff_add(A4, gx); e[2] = ff_add(A4, gy); e[3] = ff_add(A4, mgx); e[4] = ff_add(A4, mgy);
        const FF<R> sp = ff_scale(ff_add(gx, gy), R(0.25)), sm = ff_scale(ff_add(gy, mgx), R(0.25));
        e[5] = ff_add(A, sp); e[6] = ff_add(A, sm);
        e[7] = ff_add(A, FF<R>{-sp.hi, -sp.lo}); e[8] = ff_add(A, FF<R>{-sm.hi, -sm.lo});
    }
};

template <> struct ExactEqFF<D3Q7> {
    template <class R>
    __host__ __device__ static void feq(R qh, R ql, const R *Gh, const R *Gl, FF<R> *e)
    {
        const FF<R> A = {qh * R(0.125), ql * R(0.125)};
        for (int a = 0; a < 3; ++a) {
            const FF<R> h = {Gh[a] * R(0.5), Gl[a] * R(0.5)};
            e[1 + 2 * a] = ff_add(A, h);
            e[2 + 2 * a] = ff_add(A, FF<R>{-h.hi, -h.lo});
        }
    }
};
