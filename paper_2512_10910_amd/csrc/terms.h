// Device code shared by the cluster kernel and the persistent block: the
// one-thread term paths (scalar products and cycle traces) and the FP64 sum
// of a closed network's retained configurations.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pne_internal.h"
#include "regauge.h"

namespace pne {
namespace dev {

// A cycle of L sites whose cluster legs all have dimension E: the term is
// Tr(M_0 M_1 ... M_{L-1}) with M_j[a][b] the excited block of site j's slice
// (a on the leg towards site j-1, b towards site j+1).  One thread holds the
// running product (E x E) in registers.
template <int E, typename S>
__device__ inline typename SliceIO<S>::acc loop_trace(const InstStep *__restrict__ rec, int L,
                                                      const S *__restrict__ slices, int64_t base) {
    using A = typename SliceIO<S>::acc;
    A F[E][E], M[E][E];
    int xo = gld(&rec[0].xoff), x0 = gld(&rec[0].xs[0]), x1 = gld(&rec[0].xs[1]);
#pragma unroll
    for (int a = 0; a < E; ++a)
#pragma unroll
        for (int b = 0; b < E; ++b) F[a][b] = SliceIO<S>::load(slices, base + xo + a * x0 + b * x1);
    for (int j = 1; j < L; ++j) {
        xo = gld(&rec[j].xoff);
        x0 = gld(&rec[j].xs[0]);
        x1 = gld(&rec[j].xs[1]);
#pragma unroll
        for (int a = 0; a < E; ++a)
#pragma unroll
            for (int b = 0; b < E; ++b) M[a][b] = SliceIO<S>::load(slices, base + xo + a * x0 + b * x1);
        if (j == L - 1) break;
#pragma unroll
        for (int a = 0; a < E; ++a) {
            A row[E];
#pragma unroll
            for (int b = 0; b < E; ++b) {
                A acc = A(0);
#pragma unroll
                for (int c = 0; c < E; ++c) acc += F[a][c] * M[c][b];
                row[b] = acc;
            }
#pragma unroll
            for (int b = 0; b < E; ++b) F[a][b] = row[b];
        }
    }
    A tr = A(0);
#pragma unroll
    for (int a = 0; a < E; ++a)
#pragma unroll
        for (int b = 0; b < E; ++b) tr += F[a][b] * M[b][a];
    return tr;
}

// Value of one scalar or cycle instance (cd.scalar or cd.loop_e); rec are its
// step records, base the network's slice base.
template <typename S>
__device__ inline typename SliceIO<S>::acc fast_term(const ClassDesc &cd, const InstStep *__restrict__ rec,
                                                     const S *__restrict__ slices, int64_t base) {
    using A = typename SliceIO<S>::acc;
    if (cd.scalar) {
        A prod = A(1);
        for (int st = 0; st < cd.n_steps; ++st) prod *= SliceIO<S>::load(slices, base + gld(&rec[st].xoff));
        return prod;
    }
    switch (cd.loop_e) {
        case 2: return loop_trace<2, S>(rec, cd.n_verts, slices, base);
        case 3: return loop_trace<3, S>(rec, cd.n_verts, slices, base);
        case 4: return loop_trace<4, S>(rec, cd.n_verts, slices, base);
        default: return loop_trace<5, S>(rec, cd.n_verts, slices, base);
    }
}

// Sum of one value per thread over a block of NT threads, in a fixed order.
template <int NT>
__device__ inline double block_sum_nt(double v, double *red) {
    const int tid = threadIdx.x;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < NT / 64; ++k) t += red[k];
    __syncthreads();
    return t;
}

// Largest of one value per thread over a block of NT threads.
template <int NT>
__device__ inline double block_max_nt(double v, double *red) {
    const int tid = threadIdx.x;
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < NT / 64; ++k) t = fmax(t, red[k]);
    __syncthreads();
    return t;
}

// Unit roundoff of the slice precision (RNE from FP64), and of the term
// arithmetic (FP32 accumulation for FP32 and BF16 slices).
template <typename S>
__host__ __device__ constexpr double unit_roundoff() {
    return sizeof(S) == 8 ? 0x1p-53 : (sizeof(S) == 4 ? 0x1p-24 : 0x1p-8);
}
template <typename S>
__host__ __device__ constexpr double arith_roundoff() {
    return sizeof(S) == 8 ? 0x1p-53 : 0x1p-24;
}

// Per-network diagnostics by a block of NT threads (results in every thread).
//   dangling: over the network's sites without open legs and every leg l of
//     dimension d >= 2, the 2-norm of the slice entries k * stride_l,
//     k = 1..d-1 (every other leg at its vacuum index 0; the slice is the
//     regauged tensor over z'_v).  These are the single-excitation terms the
//     dangling rule drops (Sec. III.A-B); they vanish at a BP fixed point.
//   err: (sum_s ((s + 1) u + s v) A_s) (1 + A), with A_s the sum of |w|
//     over the clusters of s bonds (every entry of an open cluster's tensor)
//     and A = sum_s A_s: a first-order estimate of the error that slices
//     rounded to unit roundoff u (a term of s bonds multiplies at most s + 1
//     slices) and term arithmetic of unit roundoff v put into the sum of the
//     retained terms; the factor 1 + A covers the products of two clusters.
template <int NT, typename S>
__device__ inline void net_diagnostics(const CombineRec &cr, const GeoRec &gr, const Bucket *__restrict__ buckets,
                                       const SiteRec *__restrict__ sites, const S *__restrict__ slices,
                                       const double *__restrict__ wn, double *red, double *dangling, double *err) {
    const int tid = threadIdx.x;
    double dm = 0.0;
    for (int s = tid; s < cr.n_sites; s += NT) {
        const SiteRec *r = sites + cr.site_begin + s;
        if (gld(&r->open_mask) != 0) continue;
        const int rank = gld(&r->rank);
        const int64_t so = gld(&r->slice_off);
        for (int l = 0; l < rank; ++l) {
            const int d = gld(&r->dim[l]), st = gld(&r->stride[l]);
            double n2 = 0.0;
            for (int k = 1; k < d; ++k) {
                const double x = (double)SliceIO<S>::load(slices, so + (int64_t)k * st);
                n2 = fma(x, x, n2);
            }
            dm = fmax(dm, sqrt(n2));
        }
    }
    *dangling = block_max_nt<NT>(dm, red);
    double ws = 0.0, wt = 0.0;
    const int nb = gr.n_buckets < 64 ? gr.n_buckets : 64;
    for (int b = 0; b < nb; ++b) {
        const Bucket bk = buckets[gr.bucket_begin + b];
        const int64_t n = (int64_t)(bk.end - bk.begin) * bk.osz;
        double a = 0.0;
        for (int64_t e = tid; e < n; e += NT) a += fabs(wn[bk.w_begin + e]);
        ws = fma((bk.size + 1) * unit_roundoff<S>() + bk.size * arith_roundoff<S>(), a, ws);
        wt += a;
    }
    ws = block_sum_nt<NT>(ws, red);
    wt = block_sum_nt<NT>(wt, red);
    *err = ws * (1.0 + wt);
}

// Exponentiated form of a closed network's retained terms (one thread): the
// Mayer series of ln(1 + S) over the clusters as polymers, to second order,
//   F = sum_s W_s - 1/2 sum_{2s <= K} Q_s - (sum over overlapping pairs a < b
//       with |a| + |b| <= K of w_a w_b),
// W_s, Q_s the sum of the weights (their squares) of clusters of s bonds,
// bucket(s) the bucket of closed clusters of size s (or -1).
template <class BF>
__device__ inline double cumulant_form(const double *bw, const double *bq, BF bucket, int K, double pv) {
    double F = 0.0;
    for (int s = 1; s <= K; ++s) {
        const int b = bucket(s);
        if (b < 0) continue;
        F += bw[b];
        if (2 * s <= K) F -= 0.5 * bq[b];
    }
    return F - pv;
}

// FP64 sum of a closed network's retained configurations by a block of NT
// threads (the closed case of the combine kernel): with W_s the sum of the
// weights of clusters of size s and Q_s the sum of their squares,
//   S = sum_s W_s + sum_{s<s', s+s'<=K} W_s W_s' + sum_{2s<=K} (W_s^2 - Q_s)/2
//       - (sum over listed overlapping pairs of w_a w_b),
// ln|Z| = sum_v ln|z'_v| + ln|1 + S|; `status` is the network's status this
// run.  Also records the dangling measure and the precision estimate
// (net_diagnostics).  lds: 8 + 2*64 + 33 doubles.
template <int NT, typename S>
__device__ void combine_closed(int net, const CombineRec &cr, const GeoRec &gr, const Bucket *__restrict__ buckets,
                               const int *__restrict__ pair_a, const int *__restrict__ pair_b,
                               const PairCat *__restrict__ cats, const double *__restrict__ w,
                               const double *__restrict__ site_log, const int *__restrict__ site_sign,
                               const SiteRec *__restrict__ sites, const S *__restrict__ slices,
                               int status, NetResult *__restrict__ out, double *lds) {
    const int tid = threadIdx.x;
    double *red = lds;
    double *bw = lds + 8;
    double *bq = bw + 64;
    int *bidx = reinterpret_cast<int *>(bq + 64);
    const double *wn = w + cr.w_base;
    double lg = 0.0, neg = 0.0;
    for (int s = tid; s < cr.n_sites; s += NT) {
        lg += site_log[cr.site_begin + s];
        neg += site_sign[cr.site_begin + s] < 0 ? 1.0 : 0.0;
    }
    lg = block_sum_nt<NT>(lg, red);
    neg = block_sum_nt<NT>(neg, red);
    double dangling, err;
    net_diagnostics<NT, S>(cr, gr, buckets, sites, slices, wn, red, &dangling, &err);
    for (int i = tid; i < 33; i += NT) bidx[i] = -1;
    __syncthreads();
    const int nb = gr.n_buckets < 64 ? gr.n_buckets : 64;
    for (int b = 0; b < nb; ++b) {
        const Bucket bk = buckets[gr.bucket_begin + b];
        if (tid == 0 && bk.type == 0 && bk.size <= 32) bidx[bk.size] = b;
        double v = 0.0, q = 0.0;
        for (int c = bk.begin + tid; c < bk.end; c += NT) {
            const double x = wn[bk.w_begin + (c - bk.begin)];
            v += x;
            q = fma(x, x, q);
        }
        v = block_sum_nt<NT>(v, red);
        q = block_sum_nt<NT>(q, red);
        if (tid == 0) {
            bw[b] = v;
            bq[b] = q;
        }
    }
    double pv = 0.0;
    for (int ci = 0; ci < gr.n_pair_cats; ++ci) {
        const PairCat pc = cats[gr.pair_cat_begin + ci];
        if (pc.t1 != 0 || pc.t2 != 0) continue;
        for (int p = pc.begin + tid; p < pc.end; p += NT) {
            const int ca = pair_a[gr.pair_begin + p], cb = pair_b[gr.pair_begin + p];
            int64_t oa = -1, ob = -1;
            for (int b = 0; b < nb; ++b) {
                const Bucket bk = buckets[gr.bucket_begin + b];
                if (ca >= bk.begin && ca < bk.end) oa = bk.w_begin + (int64_t)(ca - bk.begin) * bk.osz;
                if (cb >= bk.begin && cb < bk.end) ob = bk.w_begin + (int64_t)(cb - bk.begin) * bk.osz;
            }
            pv = fma(wn[oa], wn[ob], pv);
        }
    }
    pv = block_sum_nt<NT>(pv, red);
    if (tid != 0) return;
    const int K = gr.K < 32 ? gr.K : 32;
    auto B = [&](int s) { return (s >= 0 && s <= 32) ? bidx[s] : -1; };
    double SC = 0.0;
    for (int s = 1; s <= K; ++s) {
        const int b = B(s);
        if (b >= 0) SC += bw[b];
    }
    for (int s = 1; s <= K; ++s) {
        const int b = B(s);
        if (b < 0) continue;
        for (int s2 = s + 1; s + s2 <= K; ++s2) {
            const int b2 = B(s2);
            if (b2 >= 0) SC += bw[b] * bw[b2];
        }
        if (2 * s <= K) SC += 0.5 * (bw[b] * bw[b] - bq[b]);
    }
    SC -= pv;
    NetResult res;
    res.status = status;
    res.log_bp = lg;
    res.dangling = dangling;
    const int sign_bp = ((int)neg & 1) ? -1 : 1;
    if (cr.cumulant) {
        res.sum = cumulant_form(bw, bq, B, K, pv);
        res.sign = sign_bp;
        res.log_abs = lg + res.sum;
        res.err_est = err;
        out[net] = res;
        return;
    }
    res.sum = SC;
    const double tot = 1.0 + SC;
    res.err_est = err / fabs(tot);
    res.sign = tot == 0.0 ? 0 : (tot > 0.0 ? sign_bp : -sign_bp);
    res.log_abs = lg + log(fabs(tot));
    out[net] = res;
}

}  // namespace dev
}  // namespace pne
