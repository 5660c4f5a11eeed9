// Kernel templates of the collide-and-stream library for gfx950 (MI355X)
// and the launcher template that instantiates them per (system, lattice,
// storage).  Included by one translation unit per system family
// (sys_*.hip), which the build compiles in parallel.
//
// Memory layout: structure of arrays, z-slab major: population (k, i) of
// cell (x, y, z) at [z][k][i][y][x] (for 2D grids [k][i][cells]), x fastest,
// so each wavefront of 64 lanes touches 64 consecutive cells of one
// population (fully coalesced).  A/B buffers with pull streaming: buffer P
// holds the post-collision populations of the previous step, and the
// pre-collision population of cell x is P_i(x - c_i) (periodic wrap), so
// every population crosses HBM once read and once written per step and all
// stores are aligned.
//
// One thread updates one cell: load K*Q populations (a1), moments (a2),
// fluctuation-form flux (a3), shifted equilibrium (a4), sources (a5), BGK
// relaxation (a6), aligned store (a7) -- eq. (moments), (feq) with the
// Sec. 2.5.2 shift, and (lbe_update).  The workgroup index is remapped so
// that consecutive tiles of cells run on the same XCD (the hardware
// dispatches workgroups round-robin over the 8 XCDs, each with its own L2),
// keeping the rows that neighbouring tiles share in one L2.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <type_traits>

#include "device_common.hpp"

// --------------------------------------------- manufactured forcing ----
// d_t Q + div Phi(Q) for the 3D NSF manufactured solution (exact fields of
// the homogenized-NSF MMS shape at porosity 1), conserved rows only, by
// forward-mode differentiation in (x, y, z, t) of the exact fields and of
// the flux evaluated at the exact state with exact trackers G = grad u,
// G_T = grad T (which needs the second derivatives of u and T).
template <class R>
__device__ inline void nsf_mms_source(const MmsParams<R> &m, const Phys<R> &p, R X, R Y, R Z, R *S5)
{
    using J = Dual<R, 4>;
    const R k = m.k, A = m.amp, t = m.t;
    // sin(k X) and cos(k X) for k = 2 pi and X in [0, 1): 2 X is exact and
    // sinpi / cospi reduce it exactly, where the product k X would carry a
    // rounding of up to half an ulp of 2 pi into every phase
    auto sinp = [](R v) {
        if constexpr (std::is_same<R, float>::value) return sinpif(R(2) * v);
        else return sinpi(R(2) * v);
    };
    auto cosp = [](R v) {
        if constexpr (std::is_same<R, float>::value) return cospif(R(2) * v);
        else return cospi(R(2) * v);
    };
    const R sx = sinp(X), cx = cosp(X), sy = sinp(Y), cy = cosp(Y), sz = sinp(Z), cz = cosp(Z);
    const R st = sin(t), ct = cos(t);
    // products of per-axis sines and cosines with all first derivatives
    // and the second spatial derivatives needed for the trackers
    auto trig = [&](int fx, int fy, int fz, int ft) {
        // f = Fx(kX) Fy(kY) Fz(kZ) Ft(t), F = sin (0) or cos (1)
        const R vx = fx ? cx : sx, dx_ = fx ? -k * sx : k * cx;
        const R vy = fy ? cy : sy, dy_ = fy ? -k * sy : k * cy;
        const R vz = fz ? cz : sz, dz_ = fz ? -k * sz : k * cz;
        const R vt = ft ? ct : st, dt_ = ft ? -st : ct;
        J r;
        r.v = vx * vy * vz * vt;
        r.d[0] = dx_ * vy * vz * vt;
        r.d[1] = vx * dy_ * vz * vt;
        r.d[2] = vx * vy * dz_ * vt;
        r.d[3] = vx * vy * vz * dt_;
        return r;
    };
    // exact primitives
    const J rho = trig(0, 1, 0, 1) * A + m.rho0;
    J u[3] = {trig(1, 0, 0, 0) * A + m.u0, trig(0, 1, 0, 0) * A + m.u0, trig(0, 0, 1, 0) * A + m.u0};
    const J pr = (rho - m.rho0) * m.cbar2 + trig(1, 0, 1, 0) * (A * m.p0) + m.p0;
    // conserved state as jets
    J Q[5];
    Q[0] = rho;
    for (int a = 0; a < 3; ++a) Q[1 + a] = rho * u[a];
    Q[4] = pr / (p.gamma - R(1)) + rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * R(0.5);
    // velocity gradient G_ab = d_b u_a and its spatial derivatives: u_a is
    // A * product of trig factors, so d_c d_b u_a is again such a product.
    // Build second derivatives of each u_a factor-wise.
    auto hess = [&](int fx, int fy, int fz, int b, int c) {
        // d_b d_c of Fx Fy Fz (time factor sin t applied by caller)
        R f[3] = {fx ? cx : sx, fy ? cy : sy, fz ? cz : sz};
        R df[3] = {fx ? -k * sx : k * cx, fy ? -k * sy : k * cy, fz ? -k * sz : k * cz};
        R d2f[3] = {-k * k * f[0], -k * k * f[1], -k * k * f[2]};
        R out = R(1);
        for (int a = 0; a < 3; ++a) {
            const int o = (a == b) + (a == c);
            out *= (o == 0 ? f[a] : (o == 1 ? df[a] : d2f[a]));
        }
        return out;
    };
    const int shape[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    J G[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            J g;
            g.v = u[a].d[b];
            for (int c = 0; c < 3; ++c) g.d[c] = A * st * hess(shape[a][0], shape[a][1], shape[a][2], b, c);
            g.d[3] = A * ct * hess(shape[a][0], shape[a][1], shape[a][2], b, 3);   // b != 3: first derivative only
            G[a][b] = g;
        }
    // temperature T = p / rho and its gradient with derivatives: needs the
    // Hessians of rho and p
    R Hr[3][3], Hp[3][3];
    for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c) {
            Hr[b][c] = A * ct * hess(0, 1, 0, b, c);
            Hp[b][c] = Hr[b][c] * m.cbar2 + A * m.p0 * st * hess(1, 0, 1, b, c);
        }
    J GT[3];
    {
        const R r = rho.v, P = pr.v, T = P / r;
        R gT[3];
        for (int b = 0; b < 3; ++b) gT[b] = (pr.d[b] - T * rho.d[b]) / r;
        for (int b = 0; b < 3; ++b) {
            GT[b].v = gT[b];
            for (int c = 0; c < 3; ++c)
                GT[b].d[c] = (Hp[b][c] - gT[c] * rho.d[b] - T * Hr[b][c] - gT[b] * rho.d[c]) / r;
            GT[b].d[3] = R(0);   // time derivative of the trackers is not needed
        }
    }
    // flux of the conserved rows at the exact state, tensor form
    const J ir = R(1) / rho;
    J uu[3];
    for (int a = 0; a < 3; ++a) uu[a] = Q[1 + a] * ir;
    const J pp = (Q[4] - (Q[1] * uu[0] + Q[2] * uu[1] + Q[3] * uu[2]) * R(0.5)) * (p.gamma - R(1));
    const J trG = G[0][0] + G[1][1] + G[2][2];
    J tau[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            J v = G[a][b] + G[b][a];
            if (a == b) v = v - trG * R(2.0 / 3.0);
            tau[a][b] = v * p.mu;
        }
    for (int kk = 0; kk < 5; ++kk) S5[kk] = Q[kk].d[3];
    for (int c = 0; c < 3; ++c) {
        S5[0] += Q[1 + c].d[c];
        for (int a = 0; a < 3; ++a) {
            J f = Q[1 + a] * uu[c] - tau[a][c];
            if (a == c) f = f + pp;
            S5[1 + a] += f.d[c];
        }
        J fe = (Q[4] + pp) * uu[c] - (tau[c][0] * uu[0] + tau[c][1] * uu[1] + tau[c][2] * uu[2]) - GT[c] * p.kappa;
        S5[4] += fe.d[c];
    }
}

// ---------------------------------------------------- collide & stream ----
// Workgroup size of the step kernel.  The 17-field cascade keeps ~250
// values live per cell: a 512-thread workgroup (two waves per SIMD) caps a
// wave at 256 of the SIMD's 512 registers per lane, so two waves share each
// SIMD and one hides the other's loads (in FP32 it needs 230, no spills).
// In FP64 the largest states (12 fields and more) need more than 256 even
// so and would spill to scratch; a 256-thread workgroup lets one wave per
// SIMD keep the overflow in accumulation registers instead (resistive MHD
// 1.77 -> 1.16 ms, homogenized NSF 6.07 -> 5.19 ms, 2D compressible NSF
// 778 -> 770 us per step).
template <class Sys, class St>
constexpr int step_block()
{
    return (sizeof(St) == 8 && Sys::K >= 12) ? kBlock : (Sys::K > 6 ? 512 : kBlock);
}

// Systems that form their equilibria in float-float from a plain-float
// flux deviation declare `static constexpr bool ffeq = true` (see k_step).
template <class Sys, class = void> struct FfeqOf : std::false_type {};
template <class Sys> struct FfeqOf<Sys, decltype(void(Sys::ffeq))> : std::integral_constant<bool, Sys::ffeq> {};

// collision operators of the step kernel
enum { COLL_BGK = 0, COLL_TRT = 1, COLL_REG = 2 };

template <class Sys, class Lat, class St, bool REC, bool NT, bool O32, int COLL>
__global__ __launch_bounds__((step_block<Sys, St>())) void k_step(const St *__restrict__ fin, St *__restrict__ fout,
                                                            const KParams<typename Store<St>::R> p,
                                                            typename Store<St>::R *__restrict__ qhist)
{
    using R = typename Store<St>::R;
    using I = typename Index<O32>::T;
    constexpr int K = Sys::K, Q = Lat::Q, D = Lat::D;
    constexpr int B = step_block<Sys, St>();
    constexpr I S = sizeof(St);
    // Tiles never straddle two z-planes: tile t covers the in-plane indices
    // [tp B, tp B + B) of plane z = t / tpp (tpp tiles per plane), so z and
    // the slab bases are uniform over the workgroup.
    // Tile order: XCD-contiguous runs (xcd_tile) keep the tiles that share
    // pulled rows in one L2, which pays where the grid is cache-resident
    // (plain stores), in 3D and for large states; an HBM-resident 2D step of
    // at most 300 bytes per cell update runs its tiles in dispatch order, so
    // that the eight XCDs stream one compact region of memory instead of
    // eight distant ones (2048^2: shallow water 161 -> 152.6 us, Euler 118.0
    // -> 111.7 us; 3D NSF and the 12- and 18-field systems lose 1-8% so).
    constexpr bool XCD_RUNS = !(NT && D == 2 && 2 * K * Q * sizeof(St) <= 300);
    const I P = (I)p.nx * (I)p.ny;
    const unsigned tpp = (unsigned)((P + B - 1) / B);
    const unsigned t = XCD_RUNS ? (unsigned)xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
    const int z = (int)(t / tpp);
    const I yx = (I)(t - (unsigned)z * tpp) * B + threadIdx.x;
    if (yx >= P) return;
    const I cell = (I)z * P + yx;
    const int y = (int)(yx / (I)p.nx), x = (int)(yx - (I)y * (I)p.nx);
    // byte offsets inside a slab of the tile-blocked layout: the pulled
    // population i comes from in-plane index ys nx + xs of slab zs
    I src[Q];
    int zs[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int xs = wrapi(x - Lat::cx[i], p.nx), ys = wrapi(y - Lat::cy[i], p.ny);
        zs[i] = D == 3 ? wrapi(z - Lat::cz[i], p.nz) : 0;
        src[i] = tile_offset<K, Q>((I)ys * (I)p.nx + (I)xs) * S;
    }
    const I own = tile_offset<K, Q>(yx) * S;
    const size_t slab = (size_t)K * Q * (size_t)((P + kTile - 1) / kTile * kTile);   // elements per z-slab
    // The manufactured forcing of the 3D NSF system depends on the cell's
    // coordinates and the time only: it is evaluated before the populations
    // are loaded, so that its temporaries are not live beside them.
    R Smms[5] = {R(0), R(0), R(0), R(0), R(0)};
    if constexpr (Sys::id == SYS_NSF17) {
        if (p.mms.on) {
            // the manufactured fields are periodic on the unit cube: the
            // coordinates enter reduced to [0, 1), so the sine arguments stay
            // below 2 pi on any grid (on the unit grid nothing changes)
            auto unit = [](R v) { return v - floor(v); };
            nsf_mms_source<R>(p.mms, p.phys, unit((R)x * p.mms.dx), unit((R)y * p.mms.dx), unit((R)z * p.mms.dx),
                              Smms);
        }
        __builtin_amdgcn_sched_barrier(0);
    }

    R f[K][Q];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R v = Store<St>::ld(byte_at(fin + (size_t)zs[i] * slab + (size_t)(k * Q + i) * kTile, src[i]));
            if constexpr (std::is_same<St, _Float16>::value)
                f[k][i] = v * (R)p.inv_scale[k];
            else
                f[k][i] = v;
        }
    // moments (eq. moments) by compensated summation: dQ = hi + lo exactly
    // up to the rounding of lo (two-sum of each addition).  Binary16 storage
    // sums plainly: each stored population already carries a rounding of
    // 2^-12 of its magnitude, where the FP32 sum adds ~Q 2^-24, and the
    // two-sums would be a fifth of the step's instructions.
    constexpr bool COMP = Sys::compensated && !std::is_same<St, _Float16>::value;
    R dQ[K], dQlo[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        R s = f[k][0], c = R(0);
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const R t = s + f[k][i];
            if constexpr (COMP) {
                const R bp = t - s;
                c += (s - (t - bp)) + (f[k][i] - bp);
            }
            s = t;
        }
        dQ[k] = s;
        dQlo[k] = c;
    }
    // Single-precision steppers of the precise systems evaluate the flux
    // deviation at the compensated moments: dPhi(hi) and, from one
    // forward-mode tangent, its first-order correction J(hi) lo.
    constexpr bool PRECISE = Sys::precise && !std::is_same<St, _Float16>::value;
    // per-cell coefficient field (default values when none is attached)
    using CT = CoefTraits<Sys>;
    constexpr int NB = CT::NB;
    R bl[NB > 3 ? NB : 3];
#pragma unroll
    for (int a = 0; a < (NB > 3 ? NB : 3); ++a) bl[a] = R(CT::dflt(a));
    if (p.b) {
#pragma unroll
        for (int a = 0; a < NB; ++a) bl[a] = *byte_at(p.b + a * (size_t)p.C, cell * (I)sizeof(R));
    }
    R dPhi[K][D], dPhiLo[K][D];
    static_assert(!(PRECISE && CT::in_flux), "coefficient-dependent fluxes use the plain equilibrium");
    if constexpr (CT::in_flux) {
        Sys::template flux_delta_b<R, R>(p.phys, dQ, bl, dPhi);
    } else if constexpr (PRECISE) {
        using D1 = Dual<R, 1>;
        D1 q1[K], P1[K][D];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            q1[k] = D1(dQ[k]);
            q1[k].d[0] = dQlo[k];
        }
        Sys::template flux_delta<D1, R>(p.phys, q1, P1);
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int a = 0; a < D; ++a) {
                dPhi[k][a] = P1[k][a].v;
                dPhiLo[k][a] = P1[k][a].d[0];
            }
    } else {
        Sys::template flux_delta<R, R>(p.phys, dQ, dPhi);
    }
    // Float-float equilibria: the precise systems form e = e_hi + e_lo from
    // the flux deviation and its first-order correction J(hi) lo; the large
    // tracker states (ffeq) form it from the plain-float flux deviation, the
    // exact error of lam dPhi included, which keeps the flux evaluation's
    // register budget.  The velocity-gradient trackers see the momentum's
    // rounding amplified by |u| / |du| and by 1 / (k dx) (they follow the
    // gradient of the velocity it carries): with plain-float equilibria their
    // distance to the FP64 oracle reached 3x the binary32 storage floor at
    // 128^3, with float-float ones 1.5x.
    constexpr bool FFEQ = PRECISE || (FfeqOf<Sys>::value && std::is_same<St, float>::value);
    R Sk[K];
    Sys::template source<R, R>(p.phys, dQ, bl, Sk);
    if (p.sext) {
        // explicit per-cell source (e.g. a manufactured-solution forcing
        // evaluated at t + dt/2 by the caller)
#pragma unroll
        for (int k = 0; k < K; ++k) Sk[k] += *byte_at(p.sext + k * (size_t)p.C, cell * (I)sizeof(R));
    }
    if constexpr (Sys::id == SYS_NSF17) {
#pragma unroll
        for (int k = 0; k < 5; ++k) Sk[k] += Smms[k];
    }
    // BGK relaxation post = omega feq + (1 - omega) f written as
    // post = e + c1 (e - f) with c1 = omega - 1 exactly representable (the
    // host places 2 - omega on the 2^-24 grid): e - f is exact when f is
    // within a factor two of e, so the update rounds once.  In the precise
    // path e = e_hi + e_lo and post = e_hi + (c1 (e_hi - f) + omega e_lo).
    // Two-relaxation-time (TRT): with d_i = e_i - f_i and ib the opposite
    // velocity, relaxing the symmetric and antisymmetric parts at omega+ and
    // omega- is post_i = f_i + a d_i + b d_ib, a = (omega+ + omega-)/2 (in c1
    // = a - 1 and c2 = a), b = (omega+ - omega-)/2: the BGK update plus
    // b d_ib.  Regularized: post_i = e_i + (1 - omega) w_i c_i . Pi1 / cs^2
    // with Pi1 = sum_i c_i (f_i - e_i), the non-equilibrium part projected
    // on the first-order Hermite polynomial.
    // The rest population closes the zeroth moment,
    // post_0 = f_0 + dt S + sum_{i>0} (f_i - post_i), an identity of the
    // update (the weights sum to one, the flux enters only odd moments)
    // evaluated with the stored values of post_i, so each cell's
    // post-collision moment carries a single storage rounding.
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const R c1 = p.c1[k], c2 = p.c2[k];
        R s[Q], eh[Q], el[Q];
        if constexpr (FFEQ) {
            R Gh[D], Gl[D];
            FF<R> e[Q];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                Gh[a] = p.lam * dPhi[k][a];
                if constexpr (PRECISE)
                    Gl[a] = fma(p.lam, dPhi[k][a], -Gh[a]) + p.lam * dPhiLo[k][a];
                else
                    Gl[a] = fma(p.lam, dPhi[k][a], -Gh[a]);
            }
            ExactEqFF<Lat>::feq(dQ[k], dQlo[k], Gh, Gl, e);
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                eh[i] = e[i].hi;
                el[i] = e[i].lo;
            }
        } else {
            R G[D];
#pragma unroll
            for (int a = 0; a < D; ++a) G[a] = p.lam * dPhi[k][a];
            ExactEq<Lat>::feq(dQ[k], dQlo[k], G, eh);
        }
        const R dts = p.dt * Sk[k];
        ExactEq<Lat>::zeroth(dts, s);
        R acc = dts;
        constexpr bool TRT = COLL == COLL_TRT;
        R bd[Q];                         // TRT: b d_i
        R P1[D];                         // regularized: sum_i c_i (f_i - e_i)
        if constexpr (COLL == COLL_REG) {
#pragma unroll
            for (int a = 0; a < D; ++a) P1[a] = R(0);
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                R d = f[k][i] - eh[i];
                if constexpr (FFEQ) d = d - el[i];
#pragma unroll
                for (int a = 0; a < D; ++a)
                    if (lat_c<Lat>(i, a) != 0) P1[a] = lat_c<Lat>(i, a) > 0 ? P1[a] + d : P1[a] - d;
            }
        }
        if constexpr (TRT) {
            const R tb = p.tb[k];
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                if constexpr (FFEQ)
                    bd[i] = tb * ((eh[i] - f[k][i]) + el[i]);
                else
                    bd[i] = tb * (eh[i] - f[k][i]);
            }
        }
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const R fi = f[k][i];
            R post;
            if constexpr (COLL == COLL_REG) {
                R cp = R(0);
#pragma unroll
                for (int a = 0; a < D; ++a)
                    if (lat_c<Lat>(i, a) != 0) cp = lat_c<Lat>(i, a) > 0 ? cp + P1[a] : cp - P1[a];
                // (1 - omega) w_i / cs^2 (c_i . Pi1), with w_i / cs^2 = Wn_i / Fden
                const R rg = (-c1) * (cp * (R(Lat::Wn[i]) / R(Lat::Fden)));
                if constexpr (FFEQ)
                    post = eh[i] + ((el[i] + rg) + s[i]);
                else
                    post = eh[i] + (rg + s[i]);
            } else if constexpr (TRT) {
                if constexpr (FFEQ)
                    post = eh[i] + (fma(c1, eh[i] - fi, fma(c2, el[i], bd[Lat::opp[i]])) + s[i]);
                else
                    post = fma(c1, eh[i] - fi, eh[i] + bd[Lat::opp[i]]) + s[i];
            } else if constexpr (FFEQ) {
                post = eh[i] + (fma(c1, eh[i] - fi, c2 * el[i]) + s[i]);
            } else {
                post = fma(c1, eh[i] - fi, eh[i]) + s[i];
            }
            St *dst = byte_at(fout + (size_t)z * slab + (size_t)(k * Q + i) * kTile, own);
            if constexpr (std::is_same<St, _Float16>::value) {
                const _Float16 hv = (_Float16)(post * (R)p.scale[k]);
                st_pop<NT>(dst, hv);
                post = (R)hv * (R)p.inv_scale[k];
            } else {
                Store<St>::template st<NT>(dst, post);
            }
            acc += fi - post;
        }
        R rest = f[k][0] + acc;
        if constexpr (std::is_same<St, _Float16>::value) rest *= (R)p.scale[k];
        Store<St>::template st<NT>(byte_at(fout + (size_t)z * slab + (size_t)(k * Q) * kTile, own), rest);
    }
    if constexpr (REC) {
#pragma unroll
        for (int k = 0; k < K; ++k) *byte_at(qhist + k * (size_t)p.C, cell * (I)sizeof(R)) = dQ[k];
    }
}

// ------------------------------------------------------------- init ----
// Shifted equilibrium of the given fields, in double, written in the pull
// layout: the population i of cell x lives at x - c_i.
// Flux deviation at double precision for the initialisation kernels; a
// system whose flux reads the coefficient field takes the cell's values
// (coef: [NB][C] in the stepping arithmetic type, or null for defaults).
template <class Sys, int D, class BT>
__device__ inline void init_flux_delta(const Phys<double> &ph, const double *dQ, const BT *coef, size_t C,
                                       long long cell, double dPhi[][D])
{
    using CT = CoefTraits<Sys>;
    if constexpr (CT::in_flux) {
        double bl[CT::NB];
#pragma unroll
        for (int a = 0; a < CT::NB; ++a) bl[a] = coef ? (double)coef[(size_t)a * C + cell] : CT::dflt(a);
        Sys::template flux_delta_b<double, double>(ph, dQ, bl, dPhi);
    } else {
        Sys::template flux_delta<double, double>(ph, dQ, dPhi);
    }
}

template <class Sys, class Lat, class St>
__global__ __launch_bounds__(kBlock) void k_init(const double *__restrict__ Qin, St *__restrict__ fout,
                                                 const KParams<double> p,
                                                 const typename Store<St>::R *__restrict__ coef)
{
    constexpr int K = Sys::K, Q = Lat::Q, D = Lat::D;
    const long long cell = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (cell >= p.C) return;
    int x, y, z;
    cell_coords(cell, p.nx, p.ny, x, y, z);
    long long dst[Q];
    neighbours<Lat>(x, y, z, p.nx, p.ny, p.nz, -1, dst);
    const size_t C = (size_t)p.C;
    double dQ[K], dPhi[K][D];
#pragma unroll
    for (int k = 0; k < K; ++k) dQ[k] = Qin[(size_t)k * C + cell] - p.phys.Q0[k];
    init_flux_delta<Sys, D>(p.phys, dQ, coef, C, cell, dPhi);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            double cd = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) cd += lat_c<Lat>(i, a) * dPhi[k][a];
            const double feq = Lat::w[i] * (dQ[k] + p.lam_cs2 * cd);
            Store<St>::st_init(fout + pop_at<K, Q>(k, i, dst[i], (long long)p.nx * p.ny), feq * (double)p.scale[k]);
        }
}

// per-block maxima of |f*eq_{k,i}| per field (chooses the F16 scales)
template <class Sys, class Lat, class BT>
__global__ __launch_bounds__(kBlock) void k_init_absmax(const double *__restrict__ Qin, double *__restrict__ part,
                                                        const KParams<double> p, const BT *__restrict__ coef)
{
    constexpr int K = Sys::K, Q = Lat::Q, D = Lat::D;
    __shared__ double sh[kBlock / 64];
    double mx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) mx[k] = 0.0;
    const size_t C = (size_t)p.C;
    for (long long cell = (long long)blockIdx.x * kBlock + threadIdx.x; cell < p.C;
         cell += (long long)gridDim.x * kBlock) {
        double dQ[K], dPhi[K][D];
#pragma unroll
        for (int k = 0; k < K; ++k) dQ[k] = Qin[(size_t)k * C + cell] - p.phys.Q0[k];
        init_flux_delta<Sys, D>(p.phys, dQ, coef, C, cell, dPhi);
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                double cd = 0.0;
#pragma unroll
                for (int a = 0; a < D; ++a) cd += lat_c<Lat>(i, a) * dPhi[k][a];
                const double v = fabs(Lat::w[i] * (dQ[k] + p.lam_cs2 * cd));
                mx[k] = v > mx[k] ? v : mx[k];
            }
    }
    for (int k = 0; k < K; ++k) {
        const double r = block_reduce_max(mx[k], sh);
        if (threadIdx.x == 0) part[(size_t)k * gridDim.x + blockIdx.x] = r;
    }
}

// ----------------------------------------------------------- moments ----
template <class Sys, class Lat, class St, class Out>
__global__ __launch_bounds__(kBlock) void k_moments(const St *__restrict__ fin, Out *__restrict__ out,
                                                    const KParams<double> p, int absolute)
{
    constexpr int K = Sys::K, Q = Lat::Q;
    const long long cell = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (cell >= p.C) return;
    int x, y, z;
    cell_coords(cell, p.nx, p.ny, x, y, z);
    long long src[Q];
    neighbours<Lat>(x, y, z, p.nx, p.ny, p.nz, -1, src);
    const size_t C = (size_t)p.C;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            s += (double)Store<St>::ld(fin + pop_at<K, Q>(k, i, src[i], (long long)p.nx * p.ny));
        s *= (double)p.inv_scale[k];
        out[(size_t)k * C + cell] = (Out)(absolute ? s + p.phys.Q0[k] : s);
    }
}

// -------------------------------------------------------- reductions ----
// First pass: each workgroup grid-strides over cells and writes its partial
// results [slot][block]; second pass: one workgroup combines the partials
// in a fixed order (deterministic).
template <class Sys, class Lat, class St>
__global__ __launch_bounds__(kBlock) void k_reduce1(const St *__restrict__ fin, const double *__restrict__ ref,
                                                    double *__restrict__ part, const KParams<double> p, int what)
{
    constexpr int K = Sys::K, Q = Lat::Q;
    __shared__ double sh[kBlock / 64];
    const size_t C = (size_t)p.C;
    const unsigned nb = gridDim.x;
    if (what == 4) {   // non-finite populations (the padding of a slab's last tile is not read)
        double cnt = 0.0;
        const size_t P = (size_t)p.nx * p.ny, slab = (size_t)K * Q * (size_t)padded_plane((long long)P);
        const size_t n = slab * p.nz;
        for (size_t j = (size_t)blockIdx.x * kBlock + threadIdx.x; j < n; j += (size_t)nb * kBlock) {
            const size_t r = j % slab;
            if ((r / ((size_t)K * Q * kTile)) * kTile + r % kTile >= P) continue;
            const double v = (double)Store<St>::ld(fin + j);
            cnt += isfinite(v) ? 0.0 : 1.0;
        }
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
        double q[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < Q; ++i)
                s += (double)Store<St>::ld(fin + pop_at<K, Q>(k, i, src[i], (long long)p.nx * p.ny));
            q[k] = s * (double)p.inv_scale[k] + p.phys.Q0[k];
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
            const double s = Sys::template max_speed<double>(p.phys, q);
            a0[0] = s > a0[0] ? s : a0[0];
        }
    }
    const int nslot = (what == 3) ? 1 : (what == 0 ? K : 2 * K);
    for (int j = 0; j < nslot; ++j) {
        const double v = j < K ? a0[j] : a1[j - K];
        const double r = (what == 2 || what == 3) ? block_reduce_max(v, sh) : block_reduce_sum(v, sh);
        if (threadIdx.x == 0) part[(size_t)j * nb + blockIdx.x] = r;
    }
}

static __global__ __launch_bounds__(kBlock) void k_reduce2(const double *__restrict__ part,
                                                           double *__restrict__ out, int nslot, int nb, int is_max)
{
    __shared__ double sh[kBlock / 64];
    for (int j = 0; j < nslot; ++j) {
        double v = is_max ? 0.0 : 0.0;
        for (int b = threadIdx.x; b < nb; b += kBlock) {
            const double w = part[(size_t)j * nb + b];
            v = is_max ? (w > v ? w : v) : v + w;
        }
        const double r = is_max ? block_reduce_max(v, sh) : block_reduce_sum(v, sh);
        if (threadIdx.x == 0) out[j] = r;
    }
}

// ------------------------------------------------------------ adjoint ----
// lam^n_{k,j}(x) = (1 - omega_k) mu_{k,j} + Gamma_k with mu_{k,i}(x) =
// lam^{n+1}_{k,i}(x + c_i), M0_k = sum_i w_i mu_{k,i},
// M1_{k,a} = sum_i w_i c_ia mu_{k,i} and
// Gamma_k = omega_k M0_k + (lam/cs2) sum_{k',a} omega_k' M1_{k',a} dPhi_{k',a}/dQ_k
//           + dt sum_k' M0_k' dS_k'/dQ_k,
// the transpose of d post / d f of eq. (lbe_update) (every population of a
// field enters the collision only through Q_k).  The Jacobian products come
// from one forward-mode pass with K tangents.
template <class Sys, class Lat, class R>
__global__ __launch_bounds__(kBlock) void k_adj_step(const R *__restrict__ lin, R *__restrict__ lout,
                                                     const R *__restrict__ qh, R *__restrict__ grad_b,
                                                     const KParams<R> p)
{
    constexpr int K = Sys::K, Q = Lat::Q, D = Lat::D;
    using DK = Dual<R, K>;
    const long long cell = xcd_tile(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (cell >= p.C) return;
    int x, y, z;
    cell_coords(cell, p.nx, p.ny, x, y, z);
    long long src[Q];
    neighbours<Lat>(x, y, z, p.nx, p.ny, p.nz, +1, src);
    const size_t C = (size_t)p.C;
    // This cell's moments and coefficients are loaded first, then the pulled
    // adjoint populations: the load counter retires in issue order, so the
    // Jacobian below waits only for the moments while the populations are
    // still in flight.
    DK dQ[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        dQ[k] = DK(qh[(size_t)k * C + cell]);
        dQ[k].d[k] = R(1);
    }
    R bl[3] = {R(0), R(0), R(0)};
    if (p.b) {
#pragma unroll
        for (int a = 0; a < D; ++a) bl[a] = p.b[(size_t)a * C + cell];
    }
    R mu[K][Q], M0[K], M1[K][D];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int i = 0; i < Q; ++i) mu[k][i] = lin[(size_t)(k * Q + i) * C + src[i]];
    DK dPhi[K][D], Sk[K];
    Sys::template flux_delta<DK, R>(p.phys, dQ, dPhi);
    // M0_k = sum_i w_i mu_{k,i} and L1_{k,a} = (lam/cs2) sum_i w_i c_ia mu_{k,i},
    // with integer weight numerators (powers of two) so that the moments
    // carry no constant rounding bias: M0 = (sum Wn_i mu_i)/Wden,
    // L1 = lam (sum Wn_i c_ia mu_i)/Fden.
#pragma unroll
    for (int k = 0; k < K; ++k) {
        R s0 = R(0), s1[D];
#pragma unroll
        for (int a = 0; a < D; ++a) s1[a] = R(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const R wm = (R)Lat::Wn[i] * mu[k][i];
            s0 += wm;
#pragma unroll
            for (int a = 0; a < D; ++a)
                if (lat_c<Lat>(i, a) != 0) s1[a] += (R)lat_c<Lat>(i, a) * wm;
        }
        M0[k] = s0 / (R)Lat::Wden;
#pragma unroll
        for (int a = 0; a < D; ++a) M1[k][a] = (p.lam * s1[a]) / (R)Lat::Fden;
    }
    Sys::template source<DK, R>(p.phys, dQ, bl, Sk);
    // F_k: flux and source parts of Gamma_k; the relaxation part is applied in
    // the delta form (2 M0 - mu) - delta (M0 - mu) = (1 - omega) mu + omega M0,
    // which maps a uniform adjoint field to itself exactly.
    R F[K];
#pragma unroll
    for (int k = 0; k < K; ++k) F[k] = R(0);
#pragma unroll
    for (int kp = 0; kp < K; ++kp) {
        const R wS = p.dt * M0[kp];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            R acc = wS * Sk[kp].d[k];
#pragma unroll
            for (int a = 0; a < D; ++a) acc += p.omega[kp] * M1[kp][a] * dPhi[kp][a].d[k];
            F[k] += acc;
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const R del = p.delta[k];
#pragma unroll
        for (int i = 0; i < Q; ++i)
            lout[(size_t)(k * Q + i) * C + cell] = (R(2) * M0[k] - mu[k][i]) - del * (M0[k] - mu[k][i]) + F[k];
    }
    if constexpr (Sys::id == SYS_SWE) {
        if (grad_b && p.b) {
            // S_hu_a = -g h b_a  =>  dL/db_a += dt M0_{hu_a} (-g h)
            const R h = qh[cell] + p.phys.Q0[0];
#pragma unroll
            for (int a = 0; a < 2; ++a) grad_b[(size_t)a * C + cell] += p.dt * M0[1 + a] * (-p.phys.g * h);
        }
    }
}

template <class Sys, class Lat, class R>
__global__ __launch_bounds__(kBlock) void k_adj_seed(const R *__restrict__ dLdQ, R *__restrict__ lam,
                                                     long long Cl)
{
    constexpr int K = Sys::K, Q = Lat::Q;
    const long long cell = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (cell >= Cl) return;
    const size_t C = (size_t)Cl;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const R v = dLdQ[(size_t)k * C + cell];
#pragma unroll
        for (int i = 0; i < Q; ++i) lam[(size_t)(k * Q + i) * C + cell] = v;
    }
}

// dL/dQ^0_m = M0_m + (lam/cs2) sum_{k,a} M1_{k,a} dPhi_{k,a}/dQ_m at the
// initial fields (transpose of the equilibrium initialisation), in double.
template <class Sys, class Lat, class R>
__global__ __launch_bounds__(kBlock) void k_adj_init(const R *__restrict__ lam0, const double *__restrict__ Qin,
                                                     double *__restrict__ dQ0, const KParams<double> p)
{
    constexpr int K = Sys::K, Q = Lat::Q, D = Lat::D;
    using DK = Dual<double, K>;
    const long long cell = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (cell >= p.C) return;
    const size_t C = (size_t)p.C;
    double M0[K], M1[K][D];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        M0[k] = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) M1[k][a] = 0.0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double wm = Lat::w[i] * (double)lam0[(size_t)(k * Q + i) * C + cell];
            M0[k] += wm;
#pragma unroll
            for (int a = 0; a < D; ++a) M1[k][a] += lat_c<Lat>(i, a) * wm;
        }
    }
    DK dQ[K], dPhi[K][D];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        dQ[k] = DK(Qin[(size_t)k * C + cell] - p.phys.Q0[k]);
        dQ[k].d[k] = 1.0;
    }
    Sys::template flux_delta<DK, double>(p.phys, dQ, dPhi);
#pragma unroll
    for (int m = 0; m < K; ++m) {
        double acc = M0[m];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int a = 0; a < D; ++a) acc += p.lam_cs2 * M1[k][a] * dPhi[k][a].d[m];
        dQ0[(size_t)m * C + cell] = acc;
    }
}

// -------------------------------------------------------- launchers ----
template <class Sys, class Lat, class St>
struct Impl {
    using R = typename Store<St>::R;
    static unsigned grid(long long C) { return (unsigned)((C + kBlock - 1) / kBlock); }

    template <bool REC, bool NT, bool O32, int COLL>
    static void launch_step(const lbm_state_impl &h, const void *fin, void *fout, void *qhist, hipStream_t s,
                            const KParams<R> &p)
    {
        constexpr int B = step_block<Sys, St>();
        const long long tpp = ((long long)h.nx * h.ny + B - 1) / B;    // tiles per z-plane
        hipLaunchKernelGGL((k_step<Sys, Lat, St, REC, NT, O32, COLL>), dim3((unsigned)(tpp * h.nz)), dim3(B), 0, s,
                           (const St *)fin, (St *)fout, p, (R *)qhist);
    }
    template <bool REC, bool NT, int COLL>
    static void launch_step(const lbm_state_impl &h, const void *fin, void *fout, void *qhist, hipStream_t s,
                            const KParams<R> &p)
    {
        // the 32-bit form needs one z-slab of populations and the history
        // and source planes below 4 GiB
        if (fits_o32(padded_plane((long long)h.nx * h.ny), Sys::K * Lat::Q, sizeof(St)) && fits_o32(h.C, 1, sizeof(R)))
            launch_step<REC, NT, true, COLL>(h, fin, fout, qhist, s, p);
        else
            launch_step<REC, NT, false, COLL>(h, fin, fout, qhist, s, p);
    }
    static hipError_t step(const lbm_state_impl &h, const void *fin, void *fout, void *qhist, hipStream_t s)
    {
        const double t_half = h.t0 + (h.nsteps + 0.5) * h.dt;
        const KParams<R> p = h.kparams<R>(t_half);
        const bool nt = 2 * (size_t)Sys::K * Lat::Q * sizeof(St) * (size_t)h.C > kLastLevelCacheBytes;
        const int coll = h.regularized ? COLL_REG : (h.trt_lambda > 0 ? COLL_TRT : COLL_BGK);
        if (qhist && coll != COLL_BGK) return hipErrorInvalidValue;   // the moment history serves the BGK adjoint
        if constexpr (Sys::K <= 6) {
            if (qhist) {
                nt ? launch_step<true, true, COLL_BGK>(h, fin, fout, qhist, s, p)
                   : launch_step<true, false, COLL_BGK>(h, fin, fout, qhist, s, p);
                return hipGetLastError();
            }
        } else {
            if (qhist) return hipErrorInvalidValue;   // no adjoint for the 3D cascade
        }
        if (coll == COLL_TRT)
            nt ? launch_step<false, true, COLL_TRT>(h, fin, fout, qhist, s, p)
               : launch_step<false, false, COLL_TRT>(h, fin, fout, qhist, s, p);
        else if (coll == COLL_REG)
            nt ? launch_step<false, true, COLL_REG>(h, fin, fout, qhist, s, p)
               : launch_step<false, false, COLL_REG>(h, fin, fout, qhist, s, p);
        else
            nt ? launch_step<false, true, COLL_BGK>(h, fin, fout, qhist, s, p)
               : launch_step<false, false, COLL_BGK>(h, fin, fout, qhist, s, p);
        return hipGetLastError();
    }
    static hipError_t init(const lbm_state_impl &h, const double *Q, void *fout, hipStream_t s)
    {
        const KParams<double> p = h.kparams<double>(h.t0);
        hipLaunchKernelGGL((k_init<Sys, Lat, St>), dim3(grid(h.C)), dim3(kBlock), 0, s, Q, (St *)fout, p,
                           (const R *)h.field_b);
        return hipGetLastError();
    }
    static hipError_t init_absmax(const lbm_state_impl &h, const double *Q, double *part, hipStream_t s)
    {
        const KParams<double> p = h.kparams<double>(h.t0);
        hipLaunchKernelGGL((k_init_absmax<Sys, Lat, R>), dim3(kRedBlocks), dim3(kBlock), 0, s, Q, part, p,
                           (const R *)h.field_b);
        return hipGetLastError();
    }
    static hipError_t moments(const lbm_state_impl &h, const void *fin, void *out, int absolute, int out_dtype,
                              hipStream_t s)
    {
        const KParams<double> p = h.kparams<double>(h.t0);
        if (out_dtype == 0)
            hipLaunchKernelGGL((k_moments<Sys, Lat, St, double>), dim3(grid(h.C)), dim3(kBlock), 0, s,
                               (const St *)fin, (double *)out, p, absolute);
        else
            hipLaunchKernelGGL((k_moments<Sys, Lat, St, float>), dim3(grid(h.C)), dim3(kBlock), 0, s,
                               (const St *)fin, (float *)out, p, absolute);
        return hipGetLastError();
    }
    static hipError_t reduce(const lbm_state_impl &h, const void *fin, int what, const double *ref, double *aux,
                             hipStream_t s)
    {
        const KParams<double> p = h.kparams<double>(h.t0);
        hipLaunchKernelGGL((k_reduce1<Sys, Lat, St>), dim3(kRedBlocks), dim3(kBlock), 0, s, (const St *)fin, ref,
                           aux, p, what);
        const int nslot = (what == 3 || what == 4) ? 1 : (what == 0 ? Sys::K : 2 * Sys::K);
        const int is_max = (what == 2 || what == 3) ? 1 : 0;
        hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(kBlock), 0, s, aux, aux + (size_t)2 * LBM_MAXK * kRedBlocks,
                           nslot, kRedBlocks, is_max);
        return hipGetLastError();
    }
    static hipError_t adj_seed(const lbm_state_impl &h, const void *dLdQ, void *lam, hipStream_t s)
    {
        hipLaunchKernelGGL((k_adj_seed<Sys, Lat, R>), dim3(grid(h.C)), dim3(kBlock), 0, s, (const R *)dLdQ, (R *)lam,
                           h.C);
        return hipGetLastError();
    }
    static hipError_t adj_step(const lbm_state_impl &h, const void *lin, void *lout, const void *qhist, void *gb,
                               hipStream_t s)
    {
        const KParams<R> p = h.kparams<R>(h.t0);
        hipLaunchKernelGGL((k_adj_step<Sys, Lat, R>), dim3(grid(h.C)), dim3(kBlock), 0, s, (const R *)lin, (R *)lout,
                           (const R *)qhist, (R *)gb, p);
        return hipGetLastError();
    }
    static hipError_t adj_init(const lbm_state_impl &h, const void *lam0, const double *Q, double *dQ0, hipStream_t s)
    {
        const KParams<double> p = h.kparams<double>(h.t0);
        hipLaunchKernelGGL((k_adj_init<Sys, Lat, R>), dim3(grid(h.C)), dim3(kBlock), 0, s, (const R *)lam0, Q, dQ0,
                           p);
        return hipGetLastError();
    }
    static const Launchers *get()
    {
        // the adjoint is provided for the 2D systems (K <= 6)
        if constexpr (Sys::K <= 6) {
            static const Launchers L = {Sys::K, Lat::Q, Lat::D, sizeof(St), step, init, init_absmax, moments,
                                        reduce, adj_seed, adj_step, adj_init};
            return &L;
        } else {
            static const Launchers L = {Sys::K, Lat::Q, Lat::D, sizeof(St), step, init, init_absmax, moments,
                                        reduce, nullptr, nullptr, nullptr};
            return &L;
        }
    }
};

template <class Sys, class Lat>
static const Launchers *by_storage(int storage)
{
    switch (storage) {
    case 0: return Impl<Sys, Lat, double>::get();
    case 1: return Impl<Sys, Lat, float>::get();
    case 2: return Impl<Sys, Lat, _Float16>::get();
    }
    return nullptr;
}

// Launchers of one 2D system on D2Q5 and D2Q9, for each storage; defines
// const Launchers *fn(int lat, int storage) (nullptr for other lattices).
#define LBM_DEFINE_LAUNCHERS_2D(fn, Sys)                                        \
    const Launchers *fn(int lat, int storage)                                   \
    {                                                                           \
        if (lat == LAT_D2Q5) return by_storage<Sys, D2Q5>(storage);             \
        if (lat == LAT_D2Q9) return by_storage<Sys, D2Q9>(storage);             \
        return nullptr;                                                         \
    }
