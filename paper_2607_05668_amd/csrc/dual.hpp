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

// log(1 + x) and its derivative 1 / (1 + x).
// Single precision on the device, for |x| <= 1/4, through the series
// log(1 + x) = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...), s = x / (2 + x)
// (|s| <= 1/7: five terms leave a truncation below 2^-27 of the result),
// with s carried as a float-float pair: 2 + x = t + e exactly (|x| < 2),
// s_hi = x / t by reciprocal and one Newton step, and the remainder
// x - s_hi t (exact by fma) gives s_lo = (x - s_hi t - s_hi e) / t.  The
// leading 2 s_hi is exact, so the result rounds once more than its
// correction.  About a sixth of the instructions of the library's log1pf,
// which serves larger arguments and the host.
__host__ __device__ inline float lbm_log1p(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if (!(fabsf(x) <= 0.25f)) return log1pf(x);
    const float t = 2.0f + x, e = x - (t - 2.0f);
    const float rt = __builtin_amdgcn_rcpf(t);
    float sh = x * rt;
    sh = fmaf(fmaf(-sh, t, x), rt, sh);
    const float sl = (fmaf(-sh, t, x) - sh * e) * rt;
    const float s2 = sh * sh;
    const float p = fmaf(s2, fmaf(s2, fmaf(s2, fmaf(s2, 1.0f / 11, 1.0f / 9), 1.0f / 7), 1.0f / 5), 1.0f / 3);
    return fmaf(2.0f, sh, 2.0f * fmaf(sh * s2, p, sl));
#else
    return log1pf(x);
#endif
}
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
