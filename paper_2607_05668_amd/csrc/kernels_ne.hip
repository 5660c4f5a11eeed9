// FP16 storage of the deviation from the sender's local equilibrium
// (storage LBM_F16NE).
//
// The paper stores the populations shifted by the background equilibrium
// (Sec. 2.5.2).  In binary16 that leaves a rounding of ~2^-12 |f*| per
// population per step, which over thousands of steps dominates fields that
// start at zero.  This storage keeps, for every cell y, its pre-collision
// moment deviations M(y) in FP32 and stores in binary16 only
//     g_i(y) = post_i(y) - e_i(M(y)),
// the deviation of each post-collision population from the cell's own
// (shifted, exact-moment) equilibrium e_i(M) = w_i M + (w_i/cs^2) c_i.(dt/dx)
// dPhi(M).  With post = e + (omega - 1)(e - f) + dt w_i S the stored value is
// g_i = (omega - 1)(e_i - f_i) + dt w_i S (the non-equilibrium part), formed
// without cancellation.  The receiver x = y + c_i rebuilds
//     f_i(x) = g_i(x - c_i) + e_i(M(x - c_i))
// by re-evaluating the flux at the sender's stored moments (the same float
// computation as the sender's).  Per cell update this moves K Q 2 bytes of
// populations and K 4 bytes of moments each way.
//
// Buffer layout (each of A and B): the binary16 deviations in the
// tile-blocked layout of the step kernels ([tiles][K][Q][kTile], the cells
// padded to whole tiles), padded to 256 bytes, then moments [K][cells]
// float.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "device_common.hpp"

inline size_t ne_pop_bytes(long long C, int K, int Q)
{
    return (((size_t)K * Q * (size_t)padded_plane(C) * 2) + 255) & ~(size_t)255;
}

// element offset of deviation (k, i) of cell c (2D: c = y nx + x)
template <int K, int Q>
__device__ inline size_t ne_at(int k, int i, long long c)
{
    return (size_t)tile_offset<K, Q>(c) + (size_t)(k * Q + i) * kTile;
}

// Rebuild the pre-collision populations of cell (x, y, z) from the senders'
// deviations and stored moments.
template <class Sys, class Lat>
__device__ inline void ne_load(const _Float16 *__restrict__ g, const float *__restrict__ M, const KParams<float> &p,
                               const long long *src, float f[][Lat::Q])
{
    constexpr int K = Sys::K, Q = Lat::Q, D = Lat::D;
    const size_t C = (size_t)p.C;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        float My[K], ei[K];
#pragma unroll
        for (int k = 0; k < K; ++k) My[k] = M[(size_t)k * C + src[i]];
        if (i == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) ei[k] = ExactEq<Lat>::rest(My[k]);
        } else {
            float P[K][D];
            Sys::template flux_delta<float, float>(p.phys, My, P);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                float G[D], e[Q];
#pragma unroll
                for (int a = 0; a < D; ++a) G[a] = p.lam * P[k][a];
                ExactEq<Lat>::feq(My[k], 0.0f, G, e);
                ei[k] = e[i];
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            f[k][i] = (float)g[ne_at<K, Q>(k, i, src[i])] * p.inv_scale[k] + ei[k];
    }
}

// The step works on a tile of kNeTX x kNeTY cells whose senders (the tile
// and a one-cell halo, periodic) first put the parts of their equilibrium
// into LDS: the stored moment divided by 9 (D2Q9) or 3 (D2Q5) and the two
// components of lam dPhi(M) times w_1 / cs^2 (ExactEq::parts).  The flux and
// the weight divisions of each sender are evaluated once per workgroup
// instead of once per pulled population (Q - 1 times per cell); the
// receiver finishes each pulled population's equilibrium from LDS with two
// or three operations (ExactEq::dir), bit for bit the sender-side
// definition above.
constexpr int kNeTX = 64, kNeTY = 4;

// periodic index of a halo row or column v in [-1, n + kNeTX]: one
// conditional step where the tile fits the grid, a division only on grids
// narrower than a tile
__device__ inline int pmod(int v, int n)
{
    const int r = v < 0 ? v + n : v;
    return r < n ? r : (r < 2 * n ? r - n : r % n);
}

template <class Sys, class Lat, bool NT, bool O32>
__global__ __launch_bounds__(kNeTX * kNeTY) void k_step_ne(const _Float16 *__restrict__ gin,
                                                           const float *__restrict__ Min,
                                                           _Float16 *__restrict__ gout, float *__restrict__ Mout,
                                                           const KParams<float> p)
{
    using I = typename Index<O32>::T;
    constexpr int K = Sys::K, Q = Lat::Q, D = Lat::D;
    constexpr int HX = kNeTX + 2, HY = kNeTY + 2, NH = HX * HY, NTH = kNeTX * kNeTY;
    static_assert(D == 2, "binary16 deviation storage is built for the 2D lattices");
    __shared__ float sP[K][3][NH];
    const size_t C = (size_t)p.C;
    const int tilesx = (p.nx + kNeTX - 1) / kNeTX;
    const unsigned t = (unsigned)xcd_tile(blockIdx.x, gridDim.x);
    const int tx0 = (int)(t % (unsigned)tilesx) * kNeTX, ty0 = (int)(t / (unsigned)tilesx) * kNeTY;
    const int lx = (int)threadIdx.x % kNeTX, ly = (int)threadIdx.x / kNeTX;
    const int x = tx0 + lx, y = ty0 + ly;
    const bool live = x < p.nx && y < p.ny;
    // Each thread evaluates one or two halo senders (h and h + NTH).  The
    // first sender's stored moments are loaded first, then this cell's
    // pulled binary16 deviations, which the halo work does not need: the
    // load counter retires in issue order, so the first halo flux
    // evaluation waits only for its sender's moments while the deviations
    // are still in flight.
    static_assert(NTH <= NH && NH <= 2 * NTH, "one or two halo senders per thread");
    const int h0 = (int)threadIdx.x, h1 = h0 + NTH;
    auto sender = [&](int h) {
        const int hy = h / HX, hx = h - hy * HX;
        return (size_t)pmod(ty0 + hy - 1, p.ny) * p.nx + pmod(tx0 + hx - 1, p.nx);
    };
    float M0[K];
    {
        const size_t c0 = sender(h0);
#pragma unroll
        for (int k = 0; k < K; ++k) M0[k] = Min[(size_t)k * C + c0];
    }
    // two binary16 values per register: the deviations then hold 27 of the
    // kernel's registers instead of 54 (four waves per SIMD, not three)
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    h2 gr[K][(Q + 1) / 2];
    if (live) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const I src = tile_offset<K, Q>((I)wrapi(y - Lat::cy[i], p.ny) * (I)p.nx + (I)wrapi(x - Lat::cx[i], p.nx));
#pragma unroll
            for (int k = 0; k < K; ++k) gr[k][i / 2][i % 2] = *byte_at(gin + (size_t)(k * Q + i) * kTile, src * (I)2);
        }
    }
    auto halo = [&](int h, const float *My) {
        float P[K][D];
        Sys::template flux_delta<float, float>(p.phys, My, P);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            float G[D], Pt[3];
#pragma unroll
            for (int a = 0; a < D; ++a) G[a] = p.lam * P[k][a];
            ExactEq<Lat>::parts(My[k], G, Pt);
#pragma unroll
            for (int j = 0; j < 3; ++j) sP[k][j][h] = Pt[j];
        }
    };
    halo(h0, M0);
    if (h1 < NH) {
        float M1[K];
        const size_t c1 = sender(h1);
#pragma unroll
        for (int k = 0; k < K; ++k) M1[k] = Min[(size_t)k * C + c1];
        halo(h1, M1);
    }
    __syncthreads();
    if (!live) return;                                  // no barrier follows
    const long long cell = (long long)y * p.nx + x;
    const I own = tile_offset<K, Q>((I)cell) * (I)2;
    float f[K][Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int h = (ly + 1 - Lat::cy[i]) * HX + (lx + 1 - Lat::cx[i]);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            float Pt[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) Pt[j] = sP[k][j][h];
            const float ei = i == 0 ? ExactEq<Lat>::rest_parts(Pt) : ExactEq<Lat>::dir(Pt, i);
            f[k][i] = fmaf((float)gr[k][i / 2][i % 2], p.inv_scale[k], ei);      // the scaling is exact
        }
    }
    float dQ[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float s = f[k][0];
#pragma unroll
        for (int i = 1; i < Q; ++i) s += f[k][i];
        dQ[k] = s;
    }
    float dPhi[K][D];
    Sys::template flux_delta<float, float>(p.phys, dQ, dPhi);
    float Sk[K];
    float bl[3] = {0.0f, 0.0f, 0.0f};
    if (p.b) {
#pragma unroll
        for (int a = 0; a < D; ++a) bl[a] = p.b[(size_t)a * C + cell];
    }
    Sys::template source<float, float>(p.phys, dQ, bl, Sk);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float G[D], e[Q], s[Q];
#pragma unroll
        for (int a = 0; a < D; ++a) G[a] = p.lam * dPhi[k][a];
        ExactEq<Lat>::feq(dQ[k], 0.0f, G, e);
        const float e0 = ExactEq<Lat>::rest(dQ[k]);
        const float dts = p.dt * Sk[k];
        ExactEq<Lat>::zeroth(dts, s);
        float acc = dts;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const float d = e[i] - f[k][i];
            const _Float16 hv = (_Float16)(fmaf(p.c1[k], d, s[i]) * p.scale[k]);
            st_pop<NT>(byte_at(gout + (size_t)(k * Q + i) * kTile, own), hv);
            // f - e is exactly -d and hv / scale is exact: the closure's
            // (f - e) - hv / scale is -(d + hv / scale), rounded once
            acc -= fmaf((float)hv, p.inv_scale[k], d);
        }
        const float g0 = (f[k][0] - e0) + acc;
        st_pop<NT>(byte_at(gout + (size_t)(k * Q) * kTile, own), (_Float16)(g0 * p.scale[k]));
        st_pop<NT>(Mout + (size_t)k * C + cell, dQ[k]);
    }
}

// Initial state: M(y) = Q(y) - Q0 rounded to float and, in the pull layout,
// g_i(y) = f*eq_i(Q(y + c_i)) - e_i(M(y)) with the equilibrium of the
// receiver's initial fields in double and e_i(M) as the step kernel forms it.
template <class Sys, class Lat, bool STORE>
__device__ inline void ne_init_cell(const double *__restrict__ Qin, const KParams<double> &pd,
                                    const KParams<float> &pf, long long cell, _Float16 *g, float *M, double *mx)
{
    constexpr int K = Sys::K, Q = Lat::Q, D = Lat::D;
    const size_t C = (size_t)pd.C;
    int x, y, z;
    cell_coords(cell, pd.nx, pd.ny, x, y, z);
    long long dst[Q];
    neighbours<Lat>(x, y, z, pd.nx, pd.ny, pd.nz, +1, dst);
    float My[K];
#pragma unroll
    for (int k = 0; k < K; ++k) My[k] = (float)(Qin[(size_t)k * C + cell] - pd.phys.Q0[k]);
    float Pm[K][D];
    Sys::template flux_delta<float, float>(pf.phys, My, Pm);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        // receiver's initial equilibrium in double
        double dq[K], P[K][D];
#pragma unroll
        for (int k = 0; k < K; ++k) dq[k] = Qin[(size_t)k * C + dst[i]] - pd.phys.Q0[k];
        Sys::template flux_delta<double, double>(pd.phys, dq, P);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double cd = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) cd += lat_c<Lat>(i, a) * P[k][a];
            const double feq = Lat::w[i] * (dq[k] + pd.lam_cs2 * cd);
            float ei;
            if (i == 0) {
                ei = ExactEq<Lat>::rest(My[k]);
            } else {
                float G[D], e[Q];
#pragma unroll
                for (int a = 0; a < D; ++a) G[a] = pf.lam * Pm[k][a];
                ExactEq<Lat>::feq(My[k], 0.0f, G, e);
                ei = e[i];
            }
            const double gv = feq - (double)ei;
            if constexpr (STORE)
                g[ne_at<K, Q>(k, i, cell)] = (_Float16)(gv * (double)pf.scale[k]);
            else
                mx[k] = fabs(gv) > mx[k] ? fabs(gv) : mx[k];
        }
    }
    if constexpr (STORE) {
#pragma unroll
        for (int k = 0; k < K; ++k) M[(size_t)k * C + cell] = My[k];
    }
}

template <class Sys, class Lat>
__global__ __launch_bounds__(kBlock) void k_init_ne(const double *__restrict__ Qin, _Float16 *__restrict__ g,
                                                    float *__restrict__ M, const KParams<double> pd,
                                                    const KParams<float> pf)
{
    const long long cell = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (cell >= pd.C) return;
    ne_init_cell<Sys, Lat, true>(Qin, pd, pf, cell, g, M, nullptr);
}

template <class Sys, class Lat>
__global__ __launch_bounds__(kBlock) void k_init_absmax_ne(const double *__restrict__ Qin, double *__restrict__ part,
                                                           const KParams<double> pd, const KParams<float> pf)
{
    constexpr int K = Sys::K;
    __shared__ double sh[kBlock / 64];
    double mx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) mx[k] = 0.0;
    for (long long cell = (long long)blockIdx.x * kBlock + threadIdx.x; cell < pd.C;
         cell += (long long)gridDim.x * kBlock)
        ne_init_cell<Sys, Lat, false>(Qin, pd, pf, cell, nullptr, nullptr, mx);
    for (int k = 0; k < K; ++k) {
        const double r = block_reduce_max(mx[k], sh);
        if (threadIdx.x == 0) part[(size_t)k * gridDim.x + blockIdx.x] = r;
    }
}

template <class Sys, class Lat, class Out>
__global__ __launch_bounds__(kBlock) void k_moments_ne(const _Float16 *__restrict__ g, const float *__restrict__ M,
                                                       Out *__restrict__ out, const KParams<float> p,
                                                       const KParams<double> pd, int absolute)
{
    constexpr int K = Sys::K, Q = Lat::Q;
    const long long cell = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (cell >= p.C) return;
    int x, y, z;
    cell_coords(cell, p.nx, p.ny, x, y, z);
    long long src[Q];
    neighbours<Lat>(x, y, z, p.nx, p.ny, p.nz, -1, src);
    float f[K][Q];
    ne_load<Sys, Lat>(g, M, p, src, f);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) s += (double)f[k][i];
        out[(size_t)k * (size_t)p.C + cell] = (Out)(absolute ? s + pd.phys.Q0[k] : s);
    }
}

template <class Sys, class Lat>
__global__ __launch_bounds__(kBlock) void k_reduce1_ne(const _Float16 *__restrict__ g, const float *__restrict__ M,
                                                       const double *__restrict__ ref, double *__restrict__ part,
                                                       const KParams<float> p, const KParams<double> pd, int what)
{
    constexpr int K = Sys::K, Q = Lat::Q;
    __shared__ double sh[kBlock / 64];
    const size_t C = (size_t)p.C;
    const unsigned nb = gridDim.x;
    if (what == 4) {
        double cnt = 0.0;
        // deviations in the tile-blocked layout; the padding of the last tile is never read
        const size_t n = (size_t)K * Q * (size_t)padded_plane((long long)C);
        for (size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (size_t)nb * kBlock) {
            if ((j / ((size_t)K * Q * kTile)) * kTile + j % kTile >= C) continue;
            cnt += isfinite((float)g[j]) ? 0.0 : 1.0;
        }
        for (size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x; j < (size_t)K * C; j += (size_t)nb * kBlock)
            cnt += isfinite(M[j]) ? 0.0 : 1.0;
        const double r = block_reduce_sum(cnt, sh);
        if (threadIdx.x == 0) part[blockIdx.x] = r;
        return;
    }
    double a0[K], a1[K];
#pragma unroll
    for (int k = 0; k < K; ++k) a0[k] = a1[k] = 0.0;
    for (long long cell = (long long)blockIdx.x * kBlock + threadIdx.x; cell < p.C; cell += (long long)nb * kBlock) {
        int x, y, z;
        cell_coords(cell, p.nx, p.ny, x, y, z);
        long long src[Q];
        neighbours<Lat>(x, y, z, p.nx, p.ny, p.nz, -1, src);
        float f[K][Q];
        ne_load<Sys, Lat>(g, M, p, src, f);
        double q[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i) s += (double)f[k][i];
            q[k] = s + pd.phys.Q0[k];
        }
        if (what == 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) a0[k] += q[k];
        } else if (what == 1) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double r = ref[(size_t)k * C + cell];
                a0[k] += (q[k] - r) * (q[k] - r);
                a1[k] += r * r;
            }
        } else if (what == 2) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double r = ref[(size_t)k * C + cell];
                const double e = fabs(q[k] - r);
                a0[k] = e > a0[k] ? e : a0[k];
                a1[k] = fabs(r) > a1[k] ? fabs(r) : a1[k];
            }
        } else {
            const double sp = Sys::template max_speed<double>(pd.phys, q);
            a0[0] = sp > a0[0] ? sp : a0[0];
        }
    }
    const int nslot = (what == 3) ? 1 : (what == 0 ? K : 2 * K);
    for (int j = 0; j < nslot; ++j) {
        const double v = j < K ? a0[j] : a1[j - K];
        const double r = (what == 2 || what == 3) ? block_reduce_max(v, sh) : block_reduce_sum(v, sh);
        if (threadIdx.x == 0) part[(size_t)j * nb + blockIdx.x] = r;
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce2_ne(const double *__restrict__ part, double *__restrict__ out,
                                                       int nslot, int nb, int is_max)
{
    __shared__ double sh[kBlock / 64];
    for (int j = 0; j < nslot; ++j) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nb; b += kBlock) {
            const double w = part[(size_t)j * nb + b];
            v = is_max ? (w > v ? w : v) : v + w;
        }
        const double r = is_max ? block_reduce_max(v, sh) : block_reduce_sum(v, sh);
        if (threadIdx.x == 0) out[j] = r;
    }
}

template <class Sys, class Lat>
struct ImplNE {
    static unsigned grid(long long C) { return (unsigned)((C + kBlock - 1) / kBlock); }
    static unsigned step_grid(const lbm_state_impl &h)
    {
        return (unsigned)(((h.nx + kNeTX - 1) / kNeTX) * (long long)((h.ny + kNeTY - 1) / kNeTY));
    }
    static const _Float16 *gp(const lbm_state_impl &, const void *buf) { return (const _Float16 *)buf; }
    static const float *mp(const lbm_state_impl &h, const void *buf)
    {
        return (const float *)((const char *)buf + ne_pop_bytes(h.C, Sys::K, Lat::Q));
    }

    template <bool NT, bool O32>
    static void launch(const lbm_state_impl &h, const void *fin, void *fout, const KParams<float> &p, hipStream_t s)
    {
        hipLaunchKernelGGL((k_step_ne<Sys, Lat, NT, O32>), dim3(step_grid(h)), dim3(kNeTX * kNeTY), 0, s, gp(h, fin),
                           mp(h, fin), (_Float16 *)fout, (float *)mp(h, fout), p);
    }
    static hipError_t step(const lbm_state_impl &h, const void *fin, void *fout, void *qhist, hipStream_t s)
    {
        if (qhist) return hipErrorInvalidValue;
        const KParams<float> p = h.kparams<float>(h.t0 + (h.nsteps + 0.5) * h.dt);
        const bool nt = 2 * (ne_pop_bytes(h.C, Sys::K, Lat::Q) + (size_t)Sys::K * h.C * 4) > kLastLevelCacheBytes;
        // 32-bit byte offsets when the deviations stay below 4 GiB
        const bool o32 = ne_pop_bytes(h.C, Sys::K, Lat::Q) <= 0xffffffffull;
        if (nt)
            o32 ? launch<true, true>(h, fin, fout, p, s) : launch<true, false>(h, fin, fout, p, s);
        else
            o32 ? launch<false, true>(h, fin, fout, p, s) : launch<false, false>(h, fin, fout, p, s);
        return hipGetLastError();
    }
    static hipError_t init(const lbm_state_impl &h, const double *Q, void *fout, hipStream_t s)
    {
        hipLaunchKernelGGL((k_init_ne<Sys, Lat>), dim3(grid(h.C)), dim3(kBlock), 0, s, Q, (_Float16 *)fout,
                           (float *)mp(h, fout), h.kparams<double>(h.t0), h.kparams<float>(h.t0));
        return hipGetLastError();
    }
    static hipError_t init_absmax(const lbm_state_impl &h, const double *Q, double *part, hipStream_t s)
    {
        hipLaunchKernelGGL((k_init_absmax_ne<Sys, Lat>), dim3(kRedBlocks), dim3(kBlock), 0, s, Q, part,
                           h.kparams<double>(h.t0), h.kparams<float>(h.t0));
        return hipGetLastError();
    }
    static hipError_t moments(const lbm_state_impl &h, const void *fin, void *out, int absolute, int out_dtype,
                              hipStream_t s)
    {
        const KParams<float> p = h.kparams<float>(h.t0);
        const KParams<double> pd = h.kparams<double>(h.t0);
        if (out_dtype == 0)
            hipLaunchKernelGGL((k_moments_ne<Sys, Lat, double>), dim3(grid(h.C)), dim3(kBlock), 0, s, gp(h, fin),
                               mp(h, fin), (double *)out, p, pd, absolute);
        else
            hipLaunchKernelGGL((k_moments_ne<Sys, Lat, float>), dim3(grid(h.C)), dim3(kBlock), 0, s, gp(h, fin),
                               mp(h, fin), (float *)out, p, pd, absolute);
        return hipGetLastError();
    }
    static hipError_t reduce(const lbm_state_impl &h, const void *fin, int what, const double *ref, double *aux,
                             hipStream_t s)
    {
        hipLaunchKernelGGL((k_reduce1_ne<Sys, Lat>), dim3(kRedBlocks), dim3(kBlock), 0, s, gp(h, fin), mp(h, fin), ref,
                           aux, h.kparams<float>(h.t0), h.kparams<double>(h.t0), what);
        const int nslot = (what == 3 || what == 4) ? 1 : (what == 0 ? Sys::K : 2 * Sys::K);
        const int is_max = (what == 2 || what == 3) ? 1 : 0;
        hipLaunchKernelGGL(k_reduce2_ne, dim3(1), dim3(kBlock), 0, s, aux, aux + (size_t)2 * LBM_MAXK * kRedBlocks,
                           nslot, kRedBlocks, is_max);
        return hipGetLastError();
    }
    static const Launchers *get()
    {
        static const Launchers L = {Sys::K, Lat::Q, Lat::D, 2, step, init, init_absmax, moments,
                                    reduce, nullptr, nullptr, nullptr};
        return &L;
    }
};

const Launchers *lbm_launchers_ne(int sys, int lat)
{
    switch (sys) {
    case SYS_SWE:
        if (lat == LAT_D2Q5) return ImplNE<SysSWE, D2Q5>::get();
        if (lat == LAT_D2Q9) return ImplNE<SysSWE, D2Q9>::get();
        break;
    case SYS_ADVDIFF:
        if (lat == LAT_D2Q5) return ImplNE<SysAdvDiff, D2Q5>::get();
        if (lat == LAT_D2Q9) return ImplNE<SysAdvDiff, D2Q9>::get();
        break;
    case SYS_NEOHOOKE:
        if (lat == LAT_D2Q5) return ImplNE<SysNeoHooke, D2Q5>::get();
        if (lat == LAT_D2Q9) return ImplNE<SysNeoHooke, D2Q9>::get();
        break;
    case SYS_BURGERS:
        if (lat == LAT_D2Q5) return ImplNE<SysBurgers, D2Q5>::get();
        if (lat == LAT_D2Q9) return ImplNE<SysBurgers, D2Q9>::get();
        break;
    case SYS_EULER:
        if (lat == LAT_D2Q5) return ImplNE<SysEuler, D2Q5>::get();
        if (lat == LAT_D2Q9) return ImplNE<SysEuler, D2Q9>::get();
        break;
    case SYS_MAXWELL:
        if (lat == LAT_D2Q5) return ImplNE<SysMaxwell, D2Q5>::get();
        if (lat == LAT_D2Q9) return ImplNE<SysMaxwell, D2Q9>::get();
        break;
    case SYS_ALLENCAHN:
        if (lat == LAT_D2Q5) return ImplNE<SysAllenCahn, D2Q5>::get();
        if (lat == LAT_D2Q9) return ImplNE<SysAllenCahn, D2Q9>::get();
        break;
    case SYS_RELHYDRO:
        if (lat == LAT_D2Q5) return ImplNE<SysRelHydro, D2Q5>::get();
        if (lat == LAT_D2Q9) return ImplNE<SysRelHydro, D2Q9>::get();
        break;
    case SYS_NSE:
        if (lat == LAT_D2Q5) return ImplNE<SysNSE, D2Q5>::get();
        if (lat == LAT_D2Q9) return ImplNE<SysNSE, D2Q9>::get();
        break;
    case SYS_CNSF2D:
        if (lat == LAT_D2Q5) return ImplNE<SysCNSF2D, D2Q5>::get();
        break;
    }
    return nullptr;
}
