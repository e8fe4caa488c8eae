// Device code shared by the regauge kernels and the persistent BP kernel:
// slice precision I/O, the Appendix-B bond gauge built from two messages, and
// the register-path regauge of one tile of same-shape sites.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gmem.h"
#include "pne_internal.h"

namespace pne {
namespace dev {

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Round an FP64 value to bfloat16 once (round to nearest even).  The FP32
// intermediate is truncated and carries a sticky bit, so the single rounding
// step happens at bfloat16 precision.
__device__ inline uint16_t f64_to_bf16(double x) {
    float f = __double2float_rz(x);
    uint32_t u = __float_as_uint(f);
    if ((double)f != x) u |= 1u;  // sticky
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf/nan
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

template <typename S>
struct SliceIO;
template <>
struct SliceIO<double> {
    using acc = double;
    __device__ static double load(const double *p, int64_t i) { return gld(p + i); }
    __device__ static void store(double *p, int64_t i, double v) { gst(p + i, v); }
};
template <>
struct SliceIO<float> {
    using acc = float;
    __device__ static float load(const float *p, int64_t i) { return gld(p + i); }
    __device__ static void store(float *p, int64_t i, double v) { gst(p + i, (float)v); }
};
template <>
struct SliceIO<uint16_t> {
    using acc = float;
    __device__ static float load(const uint16_t *p, int64_t i) { return bf16_to_f32(gld(p + i)); }
    __device__ static void store(uint16_t *p, int64_t i, double v) { gst(p + i, f64_to_bf16(v)); }
};


// Gauge of Appendix B for one bond slot, built from the bond's two messages.
// With a = message arriving at the bond's first site, c = message arriving at
// its second site and n = a.c, G = [a/n | R] (R = columns 1..d-1 of the
// Householder reflection that maps c/|c| onto the e0 axis, an orthonormal
// basis of c's complement) has inverse [c^T ; R^T (I - a c^T / n)].  Inserting
// G G^-1 on the bond turns P = a c^T / n into e0 e0^T, so Q keeps exactly the
// indices 1..d-1.  The first site's slot is multiplied by G, the second
// site's by the transpose of G^-1, both as T'[.k.] = sum_i T[.i.] X[i,k].
// Each endpoint site builds the transform itself (no per-bond table).
struct LegGauge {
    double inv_n, inv_nc, u0, t, ua;  // t = 2/|u|^2 with u = c/|c| - alpha e0; ua = u.a
    bool ok;                          // false: |n| ~ 0 relative to |a||c| (SINGULAR)
};

__device__ inline LegGauge leg_gauge_setup(const double *a, const double *c, int D) {
    LegGauge g;
    double n = 0.0, na = 0.0, nc = 0.0;
    for (int i = 0; i < D; ++i) {
        n = fma(a[i], c[i], n);
        na = fma(a[i], a[i], na);
        nc = fma(c[i], c[i], nc);
    }
    na = sqrt(na);
    nc = sqrt(nc);
    g.ok = (fabs(n) >= 1e-12 * na * nc) && isfinite(n) && nc > 0.0;
    g.inv_n = 1.0 / n;
    g.inv_nc = 1.0 / nc;
    const double v0 = c[0] * g.inv_nc;
    const double alpha = v0 > 0.0 ? -1.0 : 1.0;
    g.u0 = v0 - alpha;
    double uu = g.u0 * g.u0, ua = g.u0 * a[0];
    for (int i = 1; i < D; ++i) {
        const double ui = c[i] * g.inv_nc;
        uu = fma(ui, ui, uu);
        ua = fma(ui, a[i], ua);
    }
    g.t = 2.0 / uu;
    g.ua = ua;
    return g;
}

// X[i,k] of the slot transform; ak = a[k], ck = c[k], ai = a[i], ci = c[i].
__device__ inline double leg_gauge_x(const LegGauge &g, bool vside, int i, int k, double ai, double ci, double ak,
                                     double ck) {
    if (!g.ok) return i == k ? 1.0 : 0.0;
    if (k == 0) return vside ? ci : ai * g.inv_n;
    const double ui = i == 0 ? g.u0 : ci * g.inv_nc;
    const double uk = ck * g.inv_nc;
    double r = (i == k ? 1.0 : 0.0) - g.t * ui * uk;
    if (vside) r -= (ak - g.t * uk * g.ua) * g.inv_n * ci;
    return r;
}

__device__ inline void rg_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

constexpr int rg_ipow(int b, int e) { return e <= 0 ? 1 : b * rg_ipow(b, e - 1); }

// Lane layout of the register-path regauge for shape (D, R) (all R legs of
// dimension D, no open legs), as in the BP register path: the last T legs
// index lanes through power-of-two bit-fields of B bits, the first R-T legs
// index NL values held per lane; a site occupies a segment of 2^(B T) lanes.
__host__ __device__ constexpr int rg_bits(int D) { return D <= 2 ? 1 : (D <= 4 ? 2 : 3); }
__host__ __device__ constexpr int rg_lane_legs(int D, int R) { return (6 / rg_bits(D)) < R ? (6 / rg_bits(D)) : R; }
// sites per wavefront pass (one site per lane segment)
__host__ __device__ constexpr int regauge_sites_per_tile(int D, int R) {
    return 64 >> (rg_bits(D) * rg_lane_legs(D, R));
}
// LDS doubles of the slot transforms of one pass: sites * R * D^2
__host__ __device__ constexpr int rg_pass_table(int D, int R) { return regauge_sites_per_tile(D, R) * R * D * D; }
// passes per call: up to four, while the transforms fit a 512-double table
__host__ __device__ constexpr int rg_passes(int D, int R) {
    return rg_pass_table(D, R) * 4 <= 512 ? 4 : (rg_pass_table(D, R) * 2 <= 512 ? 2 : 1);
}
// sites per call and the call's LDS table (doubles)
__host__ __device__ constexpr int regauge_sites_per_call(int D, int R) {
    return rg_passes(D, R) * regauge_sites_per_tile(D, R);
}
__host__ __device__ constexpr int regauge_call_table(int D, int R) { return rg_passes(D, R) * rg_pass_table(D, R); }
constexpr int kRgXgMax = 512;

// Register-path regauge of n_sites (<= NP * sites per pass) same-shape sites
// of network `net` by one wavefront, in NP passes.  site_of(j) gives site j's
// global index and msg(o) the FP64 message value at absolute offset o; xs is
// the wavefront's LDS table (NP * pass table doubles).
//   0. every pass's tensor values are loaded first (NP loads in flight);
//   1. the slot transforms X (site, slot, D x D) go to xs, one gauge set-up
//      per (site, slot, column) spread over the lanes;
//   2. per pass: a gauge on a register leg is an in-lane mode product, on a
//      lane leg a gather of the leg's D values by shuffles; the vacuum factor
//      T'[0,...,0] (the segment's first lane) is divided out and the slice
//      stored in the term precision, ln|z'| and its sign in FP64.
template <int D, int R, typename S, int NP, typename SiteOf, typename Msg>
__device__ inline void regauge_reg(int n_sites, int net, const SiteOf &site_of, const SiteRec *__restrict__ sites,
                                   const Msg &msg, S *__restrict__ slices, double *__restrict__ site_log,
                                   int *__restrict__ site_sign, int *status, double *__restrict__ xs) {
    constexpr int B = rg_bits(D);
    constexpr int P = 1 << B;
    constexpr int T = rg_lane_legs(D, R);
    constexpr int NLEG = R - T;
    constexpr int LS = 1 << (B * T);
    constexpr int SPT = 64 / LS;
    constexpr int NL = rg_ipow(D, NLEG);
    constexpr int DT = rg_ipow(D, T);
    static_assert(NP * SPT * R * D * D <= kRgXgMax, "slot transforms exceed the LDS table");
    const int lane = threadIdx.x & 63;
    const int slot = lane / LS;
    const int tb = lane - slot * LS;
    bool inseg = true;
    int dig[T];
    int toff = 0;
#pragma unroll
    for (int m = 0; m < T; ++m) {
        dig[m] = (tb >> (B * (T - 1 - m))) & (P - 1);
        inseg = inseg && dig[m] < D;
        toff = toff * D + (dig[m] < D ? dig[m] : 0);
    }
    // 0. tensor values of every pass
    double v[NP][NL];
    int gs[NP];
    bool act[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int j = k * SPT + slot;
        act[k] = inseg && j < n_sites;
        gs[k] = site_of(j < n_sites ? j : 0);
        const double *tp = gld(&sites[gs[k]].t);
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const double x = gld(tp + q * DT + toff);  // in bounds on every lane
            v[k][q] = act[k] ? x : 0.0;
        }
    }
    rg_wave_sync();  // the wave's previous call has finished reading xs
    // 1. slot transforms, one column per item
    for (int j = lane; j < n_sites * R * D; j += 64) {
        const int s = j / (R * D);
        const int l = (j / D) % R;
        const int k = j % D;
        const SiteRec *q = sites + site_of(s);
        const bool vs = (gld(&q->vside_mask) >> l) & 1;
        const int pin = gld(&q->msg_off) + gld(&q->moff[l]);
        const int pout = gld(&q->dst[l]);
        double a[D], c[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double x = msg(pin + i), y = msg(pout + i);
            a[i] = vs ? y : x;
            c[i] = vs ? x : y;
        }
        const LegGauge g = leg_gauge_setup(a, c, D);
        if (k == 0 && !g.ok) atomicMin(status, -4);
        double ak = a[0], ck = c[0];
#pragma unroll
        for (int i = 1; i < D; ++i)
            if (k == i) {
                ak = a[i];
                ck = c[i];
            }
        double *X = xs + (s * R + l) * D * D;
#pragma unroll
        for (int i = 0; i < D; ++i) X[i * D + k] = leg_gauge_x(g, vs, i, k, a[i], c[i], ak, ck);
    }
    rg_wave_sync();
    // 2. apply and store, pass by pass
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        if (k * SPT >= n_sites) break;
        const int j = k * SPT + slot;
        const double *X0 = xs + (j < n_sites ? j : 0) * R * D * D;
        // register (lead) legs: fiber by fiber (the D values along the leg),
        // so only one fiber is held twice
#pragma unroll
        for (int kl = 0; kl < NLEG; ++kl) {
            const double *X = X0 + kl * D * D;
            const int stride = rg_ipow(D, NLEG - 1 - kl);
#pragma unroll
            for (int f = 0; f < NL / D; ++f) {
                const int q0 = (f / stride) * D * stride + f % stride;
                double fib[D];
#pragma unroll
                for (int i = 0; i < D; ++i) fib[i] = v[k][q0 + i * stride];
#pragma unroll
                for (int dk = 0; dk < D; ++dk) {
                    double acc = 0.0;
#pragma unroll
                    for (int i = 0; i < D; ++i) acc = fma(fib[i], X[i * D + dk], acc);
                    v[k][q0 + dk * stride] = acc;
                }
            }
        }
        // lane (trailing) legs
#pragma unroll
        for (int m = 0; m < T; ++m) {
            const int shift = B * (T - 1 - m);
            const int field_clear = lane & ~((P - 1) << shift);
            const double *X = X0 + (NLEG + m) * D * D;
            const int kk = dig[m] < D ? dig[m] : 0;
            double xc[D];
#pragma unroll
            for (int i = 0; i < D; ++i) xc[i] = X[i * D + kk];
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                double acc = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i) acc = fma(__shfl(v[k][q], field_clear | (i << shift), 64), xc[i], acc);
                v[k][q] = acc;
            }
        }
        // vacuum factor of each site: element 0 in the segment's first lane
        const double z = __shfl(v[k][0], slot * LS, 64);
        const bool ok = (fabs(z) > 0.0) && isfinite(z);
        if (act[k]) {
            const int64_t so = gld(&sites[gs[k]].slice_off);
            const double iz = ok ? 1.0 / z : 0.0;
#pragma unroll
            for (int q = 0; q < NL; ++q) SliceIO<S>::store(slices, so + q * DT + toff, v[k][q] * iz);
        }
        if (tb == 0 && j < n_sites) {
            gst(site_log + gs[k], ok ? log(fabs(z)) : 0.0);
            gst(site_sign + gs[k], z < 0.0 ? -1 : 1);
            if (!ok) atomicMin(status, -4);
        }
    }
}

// Register regauge for a runtime shape (all legs of dimension dc, rank
// `rank`); MULTI selects rg_passes passes per call (else one).  Shapes outside
// regauge_reg_supported are ignored.
template <typename S, bool MULTI, typename SiteOf, typename Msg>
__device__ inline void regauge_reg_any(int dc, int rank, int n_sites, int net, const SiteOf &site_of,
                                       const SiteRec *__restrict__ sites, const Msg &msg, S *__restrict__ slices,
                                       double *__restrict__ site_log, int *__restrict__ site_sign, int *status,
                                       double *__restrict__ xs) {
#define PNE_RG_CASE(D_, R_)                                                                                  \
    case D_ * 8 + R_:                                                                                       \
        regauge_reg<D_, R_, S, MULTI ? rg_passes(D_, R_) : 1>(n_sites, net, site_of, sites, msg, slices,    \
                                                               site_log, site_sign, status, xs);               \
        break;
    switch (dc * 8 + rank) {
        PNE_RG_CASE(2, 1) PNE_RG_CASE(2, 2) PNE_RG_CASE(2, 3) PNE_RG_CASE(2, 4) PNE_RG_CASE(2, 5)
        PNE_RG_CASE(2, 6) PNE_RG_CASE(3, 1) PNE_RG_CASE(3, 2) PNE_RG_CASE(3, 3) PNE_RG_CASE(3, 4)
        PNE_RG_CASE(4, 1) PNE_RG_CASE(4, 2) PNE_RG_CASE(4, 3) PNE_RG_CASE(4, 4) PNE_RG_CASE(5, 1)
        PNE_RG_CASE(5, 2) PNE_RG_CASE(6, 1) PNE_RG_CASE(6, 2)
        default: break;
    }
#undef PNE_RG_CASE
}

}  // namespace dev
}  // namespace pne
