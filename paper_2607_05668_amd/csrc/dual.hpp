// Forward-mode dual numbers with N tangent directions, used by the adjoint
// kernels to contract flux and source Jacobians (dPhi/dQ, dS/dQ) without
// hand-written derivative code.  Arithmetic is the ordinary chain rule.
#pragma once

#include <hip/hip_runtime.h>

template <class R, int N>
struct Dual {
    R v;
    R d[N];

    __host__ __device__ Dual() {}
    __host__ __device__ Dual(R x) : v(x)
    {
#pragma unroll
        for (int j = 0; j < N; ++j) d[j] = R(0);
    }
};

template <class T> struct ScalarOf { using type = T; };
template <class R, int N> struct ScalarOf<Dual<R, N>> { using type = R; };

#define DUAL_BINOP(OP, VAL, DER)                                                        \
    template <class R, int N>                                                           \
    __host__ __device__ inline Dual<R, N> operator OP(const Dual<R, N> &a, const Dual<R, N> &b) \
    {                                                                                   \
        Dual<R, N> r;                                                                   \
        r.v = VAL;                                                                      \
        _Pragma("unroll") for (int j = 0; j < N; ++j) r.d[j] = DER;                     \
        return r;                                                                       \
    }
DUAL_BINOP(+, a.v + b.v, a.d[j] + b.d[j])
DUAL_BINOP(-, a.v - b.v, a.d[j] - b.d[j])
DUAL_BINOP(*, a.v * b.v, a.d[j] * b.v + a.v * b.d[j])
#undef DUAL_BINOP

template <class R, int N>
__host__ __device__ inline Dual<R, N> operator/(const Dual<R, N> &a, const Dual<R, N> &b)
{
    Dual<R, N> r;
    const R inv = R(1) / b.v;
    r.v = a.v * inv;
#pragma unroll
    for (int j = 0; j < N; ++j) r.d[j] = (a.d[j] - r.v * b.d[j]) * inv;
    return r;
}

template <class R, int N>
__host__ __device__ inline Dual<R, N> operator-(const Dual<R, N> &a)
{
    Dual<R, N> r;
    r.v = -a.v;
#pragma unroll
    for (int j = 0; j < N; ++j) r.d[j] = -a.d[j];
    return r;
}

// mixed scalar/dual arithmetic
template <class R, int N> __host__ __device__ inline Dual<R, N> operator+(const Dual<R, N> &a, R b) { return a + Dual<R, N>(b); }
template <class R, int N> __host__ __device__ inline Dual<R, N> operator+(R a, const Dual<R, N> &b) { return Dual<R, N>(a) + b; }
template <class R, int N> __host__ __device__ inline Dual<R, N> operator-(const Dual<R, N> &a, R b) { return a - Dual<R, N>(b); }
template <class R, int N> __host__ __device__ inline Dual<R, N> operator-(R a, const Dual<R, N> &b) { return Dual<R, N>(a) - b; }
template <class R, int N>
__host__ __device__ inline Dual<R, N> operator*(const Dual<R, N> &a, R b)
{
    Dual<R, N> r;
    r.v = a.v * b;
#pragma unroll
    for (int j = 0; j < N; ++j) r.d[j] = a.d[j] * b;
    return r;
}
template <class R, int N> __host__ __device__ inline Dual<R, N> operator*(R a, const Dual<R, N> &b) { return b * a; }
template <class R, int N> __host__ __device__ inline Dual<R, N> operator/(const Dual<R, N> &a, R b) { return a * (R(1) / b); }
template <class R, int N> __host__ __device__ inline Dual<R, N> operator/(R a, const Dual<R, N> &b) { return Dual<R, N>(a) / b; }

// log(1 + x) and its derivative 1 / (1 + x)
__host__ __device__ inline float lbm_log1p(float x) { return log1pf(x); }
__host__ __device__ inline double lbm_log1p(double x) { return log1p(x); }
template <class R, int N>
__host__ __device__ inline Dual<R, N> lbm_log1p(const Dual<R, N> &a)
{
    Dual<R, N> r;
    r.v = lbm_log1p(a.v);
    const R s = R(1) / (R(1) + a.v);
#pragma unroll
    for (int j = 0; j < N; ++j) r.d[j] = a.d[j] * s;
    return r;
}

// sqrt(x) and its derivative 1 / (2 sqrt(x))
__host__ __device__ inline float lbm_sqrt(float x) { return sqrtf(x); }
__host__ __device__ inline double lbm_sqrt(double x) { return sqrt(x); }
template <class R, int N>
__host__ __device__ inline Dual<R, N> lbm_sqrt(const Dual<R, N> &a)
{
    Dual<R, N> r;
    r.v = lbm_sqrt(a.v);
    const R s = R(0.5) / r.v;
#pragma unroll
    for (int j = 0; j < N; ++j) r.d[j] = a.d[j] * s;
    return r;
}
