// Host side of the collide-and-stream library: the kernel parameters of a
// stepper (reference state, collision rates, derived reference quantities),
// the dispatch to the per-system launchers (sys_*.hip) and the bandwidth
// probes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <type_traits>

#include "device_common.hpp"

// ------------------------------------------------------ bandwidth probe --
// One 16-byte vector per thread, non-temporal both ways: the fastest plain
// copy measured on this part (the probe of achievable HBM bandwidth).
typedef float v4f __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(kBlock) void k_copy(const v4f *__restrict__ src, v4f *__restrict__ dst, size_t n4)
{
    const size_t i = (size_t)xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i < n4) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ void k_copy_tail(const unsigned char *__restrict__ src, unsigned char *__restrict__ dst, size_t n)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t lbm_launch_copy(void *dst, const void *src, size_t n, hipStream_t s)
{
    const size_t n4 = n / 16;
    if (n4) {
        const size_t nb = (n4 + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(k_copy, dim3((unsigned)nb), dim3(kBlock), 0, s, (const v4f *)src, (v4f *)dst, n4);
    }
    const size_t tail = n - n4 * 16;
    if (tail)
        hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(kBlock), 0, s, (const unsigned char *)src + n4 * 16,
                           (unsigned char *)dst + n4 * 16, tail);
    return hipGetLastError();
}

// The D2Q9 step's memory pattern without arithmetic, in the population
// layout of the step (tiles of kTile cells holding all N = 9 fields planes):
// plane j pulled from (x, y) - c_(j mod 9), periodic, and stored at (x, y).
// Like the step, a grid whose two buffers exceed the last-level cache is
// stored non-temporally, and then (at most 300 bytes per cell) its tiles
// run in dispatch order; cache-resident grids run XCD-contiguous tiles.
template <int N, bool HBM>
__global__ __launch_bounds__(kBlock) void k_streams(const float *__restrict__ src, float *__restrict__ dst, int nx,
                                                    int ny)
{
    constexpr bool XCD_RUNS = !(HBM && 2 * N * 4 <= 300);
    const unsigned P = (unsigned)nx * (unsigned)ny;
    const unsigned c = (XCD_RUNS ? (unsigned)xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x) * kBlock + threadIdx.x;
    if (c >= P) return;
    const int y = (int)(c / (unsigned)nx), x = (int)(c - (unsigned)y * nx);
    float v[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const int i = j % 9;
        const unsigned s = (unsigned)wrapi(y - D2Q9::cy[i], ny) * nx + (unsigned)wrapi(x - D2Q9::cx[i], nx);
        v[j] = *byte_at(src + (size_t)j * kTile, tile_offset<N, 1>(s) * 4u);
    }
#pragma unroll
    for (int j = 0; j < N; ++j) st_pop<HBM>(byte_at(dst + (size_t)j * kTile, tile_offset<N, 1>(c) * 4u), v[j]);
}

hipError_t lbm_launch_streams(void *dst, const void *src, int nx, int ny, int fields, hipStream_t s)
{
    const size_t P = (size_t)nx * ny;
    if (padded_plane((long long)P) * 36 * fields > 0xffffffffull) return hipErrorInvalidValue;   // 32-bit byte offsets
    const dim3 grid((unsigned)((P + kBlock - 1) / kBlock));
    const bool hbm = 2 * (size_t)padded_plane((long long)P) * 36 * fields > kLastLevelCacheBytes;
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, grid, dim3(kBlock), 0, s, (const float *)src, (float *)dst, nx, ny); };
    if (fields == 3)
        hbm ? go(k_streams<27, true>) : go(k_streams<27, false>);
    else if (fields == 6)
        hbm ? go(k_streams<54, true>) : go(k_streams<54, false>);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// The 3D D3Q7 step's memory pattern without arithmetic, in the step's
// population layout ([nz][tiles][7 F][kTile], each z-slab padded to whole
// tiles): plane j of cell (x, y, z) pulled from (x, y, z) - c_(j mod 7),
// periodic, stored at (x, y, z) with non-temporal stores.  Launched like the
// 17-field step: 512-thread workgroups over z-slab tiles in the XCD order,
// one workgroup per CU (an LDS reservation of kStreams3Lds bytes), which
// is the occupancy the step's registers allow.
constexpr int kStreams3Block = 512;
constexpr int kStreams3Lds = 96 * 1024;
template <int N>
__global__ __launch_bounds__(kStreams3Block) void k_streams3(const float *__restrict__ src, float *__restrict__ dst,
                                                           int nx, int ny, int nz)
{
    extern __shared__ float reserve[];
    const unsigned P = (unsigned)nx * (unsigned)ny;
    const unsigned tpp = (P + kStreams3Block - 1) / kStreams3Block;
    const unsigned t = (unsigned)xcd_tile(blockIdx.x, gridDim.x);
    const int z = (int)(t / tpp);
    const unsigned yx = (t - (unsigned)z * tpp) * kStreams3Block + threadIdx.x;
    if (yx >= P) return;
    const int y = (int)(yx / (unsigned)nx), x = (int)(yx - (unsigned)y * nx);
    const size_t slab = (size_t)N * (size_t)padded_plane((long long)P);
    float v[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const int i = j % 7;
        const unsigned s = (unsigned)wrapi(y - D3Q7::cy[i], ny) * nx + (unsigned)wrapi(x - D3Q7::cx[i], nx);
        const int zs = wrapi(z - D3Q7::cz[i], nz);
        v[j] = *byte_at(src + (size_t)zs * slab + (size_t)j * kTile, tile_offset<N, 1>(s) * 4u);
    }
#pragma unroll
    for (int j = 0; j < N; ++j)
        st_pop<true>(byte_at(dst + (size_t)z * slab + (size_t)j * kTile, tile_offset<N, 1>(yx) * 4u), v[j]);
    if (threadIdx.x == 0x7fffffffu) reserve[0] = v[0];      // keeps the reservation; never taken
}

hipError_t lbm_launch_streams3(void *dst, const void *src, int nx, int ny, int nz, int fields, hipStream_t s)
{
    const size_t P = (size_t)nx * ny;
    if (padded_plane((long long)P) * 28 * fields > 0xffffffffull) return hipErrorInvalidValue;   // 32-bit slab offsets
    const unsigned tpp = (unsigned)((P + kStreams3Block - 1) / kStreams3Block);
    const dim3 grid(tpp * (unsigned)nz);
    auto go = [&](auto kern) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, kStreams3Lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, grid, dim3(kStreams3Block), kStreams3Lds, s, (const float *)src, (float *)dst, nx, ny,
                           nz);
        return hipGetLastError();
    };
    if (fields == 14) return go(k_streams3<98>);
    if (fields == 17) return go(k_streams3<119>);
    return hipErrorInvalidValue;
}

// ------------------------------------------------------- host: params ----
template <class R>
KParams<R> lbm_state_impl::kparams(double t_half) const
{
    KParams<R> p;
    std::memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.C = C;
    p.lam_cs2 = (R)((dt / dx) / cs2);
    p.lam = (R)(dt / dx);
    p.dt = (R)dt;
    const double tau_grad = g_tau > 0 ? g_tau * dt : 1.0;
    for (int k = 0; k < LBM_MAXK; ++k) {
        bool trk = false;
        if (sys == SYS_ADVDIFF) trk = SysAdvDiff::tracker(k);
        if (sys == SYS_NSF17) trk = SysNSF17::tracker(k);
        if (sys == SYS_ALLENCAHN) trk = SysAllenCahn::tracker(k);
        if (sys == SYS_NSE) trk = SysNSE::tracker(k);
        if (sys == SYS_CNSF2D) trk = SysCNSF2D::tracker(k);
        if (sys == SYS_MHD) trk = SysMHD::tracker(k);
        if (sys == SYS_HCNSF) trk = SysHCNSF::tracker(k);
        if (sys >= SYS_GEN0) {
            int gd, gnc, gnp;
            lbm_gen_fields(sys - SYS_GEN0, &gd, &gnc, &gnp);
            trk = k >= gnc;
        }
        const double om = trk ? omega_t : omega_c;
        p.omega[k] = (R)om;
        p.delta[k] = (R)(2.0 - om);
        if (trt_lambda > 0) {
            const double a = trt_a[trk ? 1 : 0], b = trt_b[trk ? 1 : 0];
            p.c1[k] = (R)(a - 1.0);
            p.c2[k] = (R)a;
            p.tb[k] = (R)b;
        } else {
            p.c1[k] = (R)(om - 1.0);
            p.c2[k] = (R)om;
            p.tb[k] = R(0);
        }
        p.scale[k] = std::ldexp(1.0f, scale_exp[k]);
        p.inv_scale[k] = std::ldexp(1.0f, -scale_exp[k]);
    }
    Phys<double> d;
    std::memset(&d, 0, sizeof d);
    for (int k = 0; k < LBM_MAXK; ++k) d.Q0[k] = Q0[k];
    d.g = g;
    d.c_light = c_light;
    d.a[0] = ax;
    d.a[1] = ay;
    d.nu = nu;
    d.react = react;
    d.inv_tau_grad = 1.0 / tau_grad;
    d.gamma = gamma;
    d.mu = mu;
    d.kappa = kappa;
    d.rho0 = rho0_el;
    d.mu_s = mu_s;
    d.lam_s = lam_s;
    if (sys == SYS_NSF17 || sys == SYS_HCNSF) {
        const double r0 = Q0[0];
        double k0 = 0.0;
        for (int a = 0; a < 3; ++a) {
            d.u_ref[a] = Q0[1 + a] / r0;
            k0 += 0.5 * Q0[1 + a] * d.u_ref[a];
        }
        d.p_ref = (gamma - 1.0) * (Q0[4] - k0);
        d.T_ref = d.p_ref / r0;
        d.H_ref = Q0[4] + d.p_ref;
        if (sys == SYS_NSF17) {
            const double trG = Q0[5] + Q0[9] + Q0[13];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    d.tau_ref[3 * a + b] =
                        mu * (Q0[5 + 3 * a + b] + Q0[5 + 3 * b + a] - (a == b ? 2.0 / 3.0 * trG : 0.0));
        }
    }
    if (sys == SYS_SWE || sys == SYS_EULER || sys == SYS_NSE) {
        d.mm0_h0[0] = Q0[1] * Q0[1] / Q0[0];
        d.mm0_h0[1] = Q0[1] * Q0[2] / Q0[0];
        d.mm0_h0[2] = Q0[2] * Q0[2] / Q0[0];
    }
    if (sys == SYS_RELHYDRO) {
        d.sq_ref = std::sqrt(4.0 * Q0[0] * Q0[0] - 3.0 * (Q0[1] * Q0[1] + Q0[2] * Q0[2]));
        d.p_ref = (d.sq_ref - Q0[0]) / 3.0;
        d.H_ref = Q0[0] + d.p_ref;
        d.mm0_h0[0] = Q0[1] * Q0[1] / d.H_ref;
        d.mm0_h0[1] = Q0[1] * Q0[2] / d.H_ref;
        d.mm0_h0[2] = Q0[2] * Q0[2] / d.H_ref;
    }
    if (sys == SYS_MHD) {
        const double b2 = Q0[4] * Q0[4] + Q0[5] * Q0[5];
        d.p_ref = (gamma - 1.0) * (Q0[3] - 0.5 * (Q0[1] * Q0[1] + Q0[2] * Q0[2]) / Q0[0] - 0.5 * b2);
        d.H_ref = Q0[3] + d.p_ref + 0.5 * b2;        // E0 + p_tot0
        for (int a = 0; a < 2; ++a) d.u_ref[a] = Q0[1 + a] / Q0[0];
    }
    d.cs2_phys = cs_phys * cs_phys;
    d.inv_R_gas = 1.0 / R_gas;
    d.inv_eta = 1.0 / eta_drag;
    if (sys >= SYS_GEN0)
        for (int j = 0; j < 16; ++j) d.gen[j] = gen_par[j];
    if (sys == SYS_EULER || sys == SYS_CNSF2D) {
        d.p_ref = (gamma - 1.0) * (Q0[3] - 0.5 * (Q0[1] * Q0[1] + Q0[2] * Q0[2]) / Q0[0]);
        d.H_ref = Q0[3] + d.p_ref;
        for (int a = 0; a < 2; ++a) {
            d.u_ref[a] = Q0[1 + a] / Q0[0];
            d.Hu_ref[a] = d.H_ref * Q0[1 + a] / Q0[0];
        }
    }
    if (sys == SYS_NEOHOOKE) {
        double H[4] = {Q0[0] - 1.0, Q0[1], Q0[2], Q0[3] - 1.0}, P[4];
        for (int j = 0; j < 4; ++j) d.H0[j] = H[j];
        SysNeoHooke::stress<double, double>(d, H, P);
        for (int j = 0; j < 4; ++j) d.P0[j] = P[j];
    }
    // convert
    for (int k = 0; k < LBM_MAXK; ++k) p.phys.Q0[k] = (R)d.Q0[k];
    p.phys.g = (R)d.g;
    p.phys.c_light = (R)d.c_light;
    p.phys.cs2_phys = (R)d.cs2_phys;
    p.phys.sq_ref = (R)d.sq_ref;
    p.phys.inv_R_gas = (R)d.inv_R_gas;
    p.phys.inv_eta = (R)d.inv_eta;
    for (int j = 0; j < 16; ++j) p.phys.gen[j] = (R)d.gen[j];
    for (int j = 0; j < 3; ++j) {
        p.phys.mm0_h0[j] = (R)d.mm0_h0[j];
        p.phys.Hu_ref[j] = (R)d.Hu_ref[j];
    }
    for (int a = 0; a < 3; ++a) {
        p.phys.a[a] = (R)d.a[a];
        p.phys.u_ref[a] = (R)d.u_ref[a];
    }
    p.phys.nu = (R)d.nu;
    p.phys.react = (R)d.react;
    p.phys.inv_tau_grad = (R)d.inv_tau_grad;
    p.phys.gamma = (R)d.gamma;
    p.phys.mu = (R)d.mu;
    p.phys.kappa = (R)d.kappa;
    p.phys.p_ref = (R)d.p_ref;
    p.phys.T_ref = (R)d.T_ref;
    p.phys.H_ref = (R)d.H_ref;
    for (int j = 0; j < 9; ++j) p.phys.tau_ref[j] = (R)d.tau_ref[j];
    p.phys.rho0 = (R)d.rho0;
    p.phys.mu_s = (R)d.mu_s;
    p.phys.lam_s = (R)d.lam_s;
    for (int j = 0; j < 4; ++j) {
        p.phys.H0[j] = (R)d.H0[j];
        p.phys.P0[j] = (R)d.P0[j];
    }
    p.b = (const R *)field_b;
    p.sext = (const R *)field_src;
    p.mms.on = (sys == SYS_NSF17) ? mms_on : 0;
    p.mms.amp = (R)mms_amp;
    p.mms.rho0 = (R)mms_rho0;
    p.mms.p0 = (R)mms_p0;
    p.mms.u0 = (R)mms_u0;
    p.mms.cbar2 = (R)(gamma * mms_p0 / mms_rho0);
    p.mms.t = (R)t_half;
    p.mms.k = (R)(2.0 * 3.14159265358979323846);
    p.mms.dx = (R)dx;
    return p;
}

const Launchers *lbm_launchers(int sys, int lat, int storage)
{
    if (storage == 3) return lbm_launchers_ne(sys, lat);
    switch (sys) {
    case SYS_SWE: return lbm_launchers_swe(lat, storage);
    case SYS_ADVDIFF: return lbm_launchers_advdiff(lat, storage);
    case SYS_NEOHOOKE: return lbm_launchers_neohooke(lat, storage);
    case SYS_NSF17: return lbm_launchers_nsf17(lat, storage);
    case SYS_BURGERS: return lbm_launchers_burgers(lat, storage);
    case SYS_EULER: return lbm_launchers_euler(lat, storage);
    case SYS_MAXWELL: return lbm_launchers_maxwell(lat, storage);
    case SYS_ALLENCAHN: return lbm_launchers_allencahn(lat, storage);
    case SYS_RELHYDRO: return lbm_launchers_relhydro(lat, storage);
    case SYS_NSE: return lbm_launchers_nse(lat, storage);
    case SYS_CNSF2D: return lbm_launchers_cnsf2d(lat, storage);
    case SYS_MHD: return lbm_launchers_mhd(lat, storage);
    case SYS_HCNSF: return lbm_launchers_hcnsf(lat, storage);
    default:
        if (sys >= SYS_GEN0) return lbm_launchers_gen(sys - SYS_GEN0, lat, storage);
    }
    return nullptr;
}

template KParams<float> lbm_state_impl::kparams<float>(double) const;
template KParams<double> lbm_state_impl::kparams<double>(double) const;
