// gfx950 kernels of the partitioned network expansion hot path.
//
//   (BP sweeps live in bp.hip)
//   k_regauge   per site: build each bond's rank-1 projector from its two
//               messages in the symmetrising gauge of Appendix B (P = e0 e0^T,
//               Q = the rest), apply it, split off the vacuum factor and store
//               the excited slices in the term precision
//   k_clusters  per cluster instance: contract the excited slices (the loop
//               terms of Sec. III.A-B; every term keeps the original geometry
//               with modified tensors, Sec. VI)
//   k_combine   per network: FP64 sum of the retained configurations
//               (Eq. (4) truncated to degree <= K, vertex-disjoint products)
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "pne.h"
#include "regauge.h"
#include "terms.h"

namespace pne {

namespace {

using namespace dev;

constexpr int kRgThreads = 128;
constexpr int kClThreads = 256;
constexpr int kCbThreads = 256;


// Per site (one block): build the gauge of every bond slot, apply them (mode
// products in LDS), then divide by the vacuum factor z'_v = T'[0,...,0] (closed sites) or
// by the largest magnitude of the vacuum vector (sites with open legs), and
// store the result in the slice precision.  ln|z'| and its sign are kept in
// FP64; their sum over sites is ln|Z_BP|.
// One mode product of the staged site tensor along a leg of dimension DD and
// stride sl: each thread takes whole fibers (the DD entries along the leg),
// reads them once and writes the DD outputs, with the same summation order
// as the per-entry form below.  Fibers are disjoint, so b1 may be b0.
template <int DD>
__device__ inline void mode_product_fibers(const double *b0, double *b1, const double *s_x, int size, int sl) {
    const int nf = size / DD;
    for (int f = threadIdx.x; f < nf; f += kRgThreads) {
        const int hi = f / sl;
        const int base = hi * DD * sl + (f - hi * sl);
        double xin[DD];
#pragma unroll
        for (int i = 0; i < DD; ++i) xin[i] = b0[base + i * sl];
#pragma unroll
        for (int k = 0; k < DD; ++k) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < DD; ++i) acc = fma(xin[i], s_x[i * DD + k], acc);
            b1[base + k * sl] = acc;
        }
    }
}

// One column k of a slot transform X (d x d, row-major) for a leg of
// dimension DD: the two messages are read into registers with every load in
// flight at once, then the gauge is built from them (the same arithmetic as
// the loop over a runtime dimension, which waits on each message load in
// turn).
template <int DD>
__device__ inline void slot_column(const double *pa, const double *pc, bool vs, int k, double *X, int *status) {
    double a[DD], c[DD];
#pragma unroll
    for (int i = 0; i < DD; ++i) {
        a[i] = pa[i];
        c[i] = pc[i];
    }
    const LegGauge g = leg_gauge_setup(a, c, DD);
    if (k == 0 && !g.ok) atomicMin(status, -4);
    double ak = a[0], ck = c[0];
#pragma unroll
    for (int i = 1; i < DD; ++i)
        if (k == i) {
            ak = a[i];
            ck = c[i];
        }
#pragma unroll
    for (int i = 0; i < DD; ++i) X[i * DD + k] = leg_gauge_x(g, vs, i, k, a[i], c[i], ak, ck);
}

template <typename S>
__global__ void __launch_bounds__(kRgThreads)
k_regauge(const SiteRec *__restrict__ sites,
                                                        const int *__restrict__ rg_sites,
                                                        const double *msg0, const double *msg1,
                                                        S *__restrict__ slices,
                                                        double *__restrict__ site_log, int *__restrict__ site_sign,
                                                        double *__restrict__ vac, NetState *st) {
    const int gsite = rg_sites[blockIdx.x];
    extern __shared__ double lds[];
    __shared__ double s_norm;
    __shared__ int s_ok;
    // the site record and the slot transforms' offsets in LDS: indexed by
    // slot at run time, they would otherwise live in scratch
    __shared__ SiteRec s_rec;
    __shared__ int xoff[kMaxRank];
    const int tid = threadIdx.x;
    if (tid < (int)(sizeof(SiteRec) / 4))
        reinterpret_cast<int *>(&s_rec)[tid] = gld(reinterpret_cast<const int *>(sites + gsite) + tid);
    __syncthreads();
    const SiteRec &r = s_rec;
    if (tid == 0) {
        int o = 0;
        for (int l = 0; l < r.rank; ++l) {
            xoff[l] = o;
            if (!((r.open_mask >> l) & 1)) o += r.dim[l] * r.dim[l];
        }
    }
    const int size = r.size;
    // legs of dimension <= 6 take the fiber-wise product, in place; larger
    // ones the per-entry form, which needs a second buffer
    const int nbuf = regauge_site_buffers(r);
    double *b0 = lds;
    double *b1 = lds + (nbuf - 1) * size;
    double *xt = lds + nbuf * size;  // the slot transforms, d_l x d_l each (regauge_site_lds_doubles)
    const double *mb = st[r.net].parity ? msg1 : msg0;
    // the tensor's first 12 * kRgThreads entries go to registers first (one
    // load round for sites of up to 1536 entries) ...
    double tv[12];
#pragma unroll
    for (int u = 0; u < 12; ++u) {
        const int e = tid + u * kRgThreads;
        tv[u] = e < size ? gld(r.t + e) : 0.0;
    }
    // ... while every slot's transform is built (one column per thread), so
    // the message loads are in flight together with the tensor's
    for (int it = tid; it < r.rank * kMaxDim; it += kRgThreads) {
        const int l = it / kMaxDim, k = it - l * kMaxDim;
        const int d = r.dim[l];
        if (k >= d || ((r.open_mask >> l) & 1)) continue;
        int xo = 0;  // this slot's transform offset (thread 0 tabulates them for later)
        for (int l2 = 0; l2 < l; ++l2)
            if (!((r.open_mask >> l2) & 1)) xo += r.dim[l2] * r.dim[l2];
        const bool vs = (r.vside_mask >> l) & 1;
        const double *pin = mb + r.msg_off + r.moff[l];
        const double *pout = mb + r.dst[l];
        const double *pa = vs ? pout : pin;
        const double *pc = vs ? pin : pout;
        double *X = xt + xo;
        switch (d) {
            case 2: slot_column<2>(pa, pc, vs, k, X, &st[r.net].status); break;
            case 3: slot_column<3>(pa, pc, vs, k, X, &st[r.net].status); break;
            case 4: slot_column<4>(pa, pc, vs, k, X, &st[r.net].status); break;
            case 5: slot_column<5>(pa, pc, vs, k, X, &st[r.net].status); break;
            case 6: slot_column<6>(pa, pc, vs, k, X, &st[r.net].status); break;
            default: {
                const LegGauge g = leg_gauge_setup(pa, pc, d);
                if (k == 0 && !g.ok) atomicMin(&st[r.net].status, -4);
                for (int i = 0; i < d; ++i) X[i * d + k] = leg_gauge_x(g, vs, i, k, pa[i], pc[i], pa[k], pc[k]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 12; ++u) {
        const int e = tid + u * kRgThreads;
        if (e < size) b0[e] = tv[u];
    }
    for (int e = tid + 12 * kRgThreads; e < size; e += kRgThreads) b0[e] = gld(r.t + e);
    __syncthreads();
    for (int l = 0; l < r.rank; ++l) {
        const int d = r.dim[l];
        if ((r.open_mask >> l) & 1) continue;
        const double *s_x = xt + xoff[l];
        const int sl = r.stride[l];
        switch (d) {
            case 2: mode_product_fibers<2>(b0, b1, s_x, size, sl); break;
            case 3: mode_product_fibers<3>(b0, b1, s_x, size, sl); break;
            case 4: mode_product_fibers<4>(b0, b1, s_x, size, sl); break;
            case 5: mode_product_fibers<5>(b0, b1, s_x, size, sl); break;
            case 6: mode_product_fibers<6>(b0, b1, s_x, size, sl); break;
            default:
                for (int e = tid; e < size; e += kRgThreads) {
                    const int k = (e / sl) % d;
                    const int base = e - k * sl;
                    double acc = 0.0;
                    for (int i = 0; i < d; ++i) acc = fma(b0[base + i * sl], s_x[i * d + k], acc);
                    b1[e] = acc;
                }
        }
        __syncthreads();
        double *t = b0;
        b0 = b1;
        b1 = t;
    }
    if (tid == 0) {
        double nv;
        int sg = 1;
        if (r.open_mask == 0) {
            nv = b0[0];
            sg = nv < 0.0 ? -1 : 1;
        } else {
            // vacuum vector over the open legs (bond indices 0)
            int n_open = 1;
            for (int l = 0; l < r.rank; ++l)
                if ((r.open_mask >> l) & 1) n_open *= r.dim[l];
            nv = 0.0;
            for (int p = 0; p < n_open; ++p) {
                int rem = p, off = 0;
                for (int l = r.rank - 1; l >= 0; --l) {
                    if (!((r.open_mask >> l) & 1)) continue;
                    off += (rem % r.dim[l]) * r.stride[l];
                    rem /= r.dim[l];
                }
                nv = fmax(nv, fabs(b0[off]));
            }
        }
        s_ok = (fabs(nv) > 0.0) && isfinite(nv);
        s_norm = nv;
        site_log[gsite] = s_ok ? log(fabs(nv)) : 0.0;
        site_sign[gsite] = sg;
        if (!s_ok) atomicMin(&st[r.net].status, -4);
    }
    __syncthreads();
    if (!s_ok) return;
    const double nv = s_norm;
    for (int e = tid; e < size; e += kRgThreads) SliceIO<S>::store(slices, r.slice_off + e, b0[e] / nv);
    if (r.open_mask != 0) {
        int n_open = 1;
        for (int l = 0; l < r.rank; ++l)
            if ((r.open_mask >> l) & 1) n_open *= r.dim[l];
        for (int p = tid; p < n_open; p += kRgThreads) {
            int rem = p, off = 0;
            for (int l = r.rank - 1; l >= 0; --l) {
                if (!((r.open_mask >> l) & 1)) continue;
                off += (rem % r.dim[l]) * r.stride[l];
                rem /= r.dim[l];
            }
            vac[r.vac_off + p] = b0[off] / nv;
        }
    }
}

struct GlobalMsg {
    const double *mb;
    __device__ double operator()(int o) const { return mb[o]; }
};

template <typename S>
__global__ void __launch_bounds__(64) k_regauge_tiles(const BpTile *__restrict__ tiles, const int *__restrict__ rg_tiles,
                                                      const SiteRec *__restrict__ sites,
                                                      const int *__restrict__ tile_sites, const double *msg0,
                                                      const double *msg1, S *__restrict__ slices,
                                                      double *__restrict__ site_log,
                                                      int *__restrict__ site_sign, NetState *st) {
    const BpTile tl = tiles[rg_tiles[blockIdx.x]];
    __shared__ double s_xg[kRgXgMax];
    const GlobalMsg msg{st[tl.net].parity ? msg1 : msg0};
    const int *ts = tile_sites + tl.site_begin;
    auto site_of = [ts](int j) { return ts[j]; };
    regauge_reg_any<S, false>(tl.dc, tl.rank, tl.n_sites, tl.net, site_of, sites, msg, slices, site_log, site_sign,
                              &st[tl.net].status, s_xg);
}

// Register-path regauge of the shapes whose lead legs hold 5 to 16 values per
// lane (rank 3 at D = 5, 6; rank 5 at D = 3, 4), one site per wavefront.  The
// persistent kernel keeps to at most 4 values per lane for its registers;
// these kernels run alone, one per shape (80-110 VGPRs).  Rank 4 at D = 5, 6
// and rank 6 at D = 3 (25-36 values per lane) stay on the per-site LDS
// kernel: in this form rank 4 at D = 6 takes 256 VGPRs and 186 AGPRs (one
// wave per SIMD) and was slower than the LDS kernel on 32x32 D = 6 networks
// (1.89 against 1.44 ms for 131k sites); capped at two waves it spills.
template <int D, int R, typename S>
__global__ void __launch_bounds__(64) k_regauge_wide(const BpTile *__restrict__ tiles, const int *__restrict__ rg_wide,
                                                     const SiteRec *__restrict__ sites,
                                                     const int *__restrict__ tile_sites, const double *msg0,
                                                     const double *msg1, S *__restrict__ slices,
                                                     double *__restrict__ site_log, int *__restrict__ site_sign,
                                                     NetState *st) {
    const BpTile tl = tiles[rg_wide[blockIdx.x]];
    __shared__ double s_xg[kRgXgMax];
    const GlobalMsg msg{st[tl.net].parity ? msg1 : msg0};
    const int *ts = tile_sites + tl.site_begin;
    auto site_of = [ts](int j) { return ts[j]; };
    regauge_reg<D, R, S, 1>(tl.n_sites, tl.net, site_of, sites, msg, slices, site_log, site_sign,
                            &st[tl.net].status, s_xg);
}

// Logical block of a physical one so that consecutive logical blocks run on
// the same XCD (workgroups are dealt to the eight XCDs round robin): blocks
// of one network, which read the same slices, then share that XCD's L2.
__device__ inline int xcd_block(int p, int nb) {
    const int x = p & 7, q = nb >> 3, r = nb & 7;
    return x * q + min(x, r) + (p >> 3);
}

// Slice offset of a StepEnt's digits (4 bits per slice leg) under an
// instance's leg strides (below 2^24: the plan tables check it).
__device__ __forceinline__ int ent_offset(uint32_t xdig, const int (&xs)[kMaxLab]) {
    unsigned x = 0;
#pragma unroll
    for (int m = 0; m < kMaxLab; ++m) x += __umul24((xdig >> (4 * m)) & 15u, (unsigned)xs[m]);
    return (int)x;
}

// Index check of the checked build (PNE_CHECKED): an index outside [0, n)
// is noted in bad and replaced by 0, so the access stays inside its buffer
// and the network reports PNE_ERR_CHECK.  Without PNE_CHECKED it is the
// index itself.
__device__ __forceinline__ int64_t chk(int64_t i, int64_t n, bool &bad) {
#ifdef PNE_CHECKED
    const bool ok = i >= 0 && i < n;
    bad = bad || !ok;
    return ok ? i : 0;
#else
    (void)n;
    (void)bad;
    return i;
#endif
}

// acc + sum over N consecutive summed entries q of F[fb + q.x] *
// slices[xb + q.y], in order, with all N loads issued before the first
// product.
template <int N, typename A, typename S>
__device__ __forceinline__ A sum_entries(A acc, const int2 *q, const A *F, int fb, int max_f, const S *slices,
                                         int64_t xb, int64_t n_slices, bool &bad) {
    A fv[N], xv[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int2 e = q[i];
        xv[i] = SliceIO<S>::load(slices, chk(xb + e.y, n_slices, bad));
        fv[i] = F[chk(fb + e.x, max_f, bad)];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) acc += fv[i] * xv[i];
    return acc;
}

// Orders the LDS accesses of the lanes of one wavefront (an instance's lanes
// never span two wavefronts: the group size divides 64).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cluster contraction by a per-class plan: the frontier tensor F absorbs one
// excited slice per step (F_next[out] = sum_shared F[.] X[.]).  A class runs
// `group` lanes per instance; every step is uniform across the block.  An
// instance's step records (slice offset from its network's slice base, leg
// strides) come from the plan's instance table; classes whose frontier has
// one entry throughout are a plain product of one slice element per vertex,
// one instance per thread.  Classes with entry tables (max_sum > 0) read
// each output's and each summed entry's F offset and slice digits from
// them; the instance's lanes first turn the summed entries into (F, slice)
// offset pairs in LDS, then each lane sums its outputs over them, in the
// same order as the index walk of the other classes.  KIND selects the
// blocks' path (0 frontier plans, 1-4 cycles of leg dimension KIND + 1, 5
// scalar products): each path is its own launch, so one path's registers
// (a dimension-5 cycle's matrices) do not lower the occupancy of another.
// n_slices, n_w and n_ents are the extents the checked build tests indices
// against; st receives its PNE_ERR_CHECK.
template <typename S, int KIND>
__global__ void __launch_bounds__(kClThreads) k_clusters(
    const ClassDesc *__restrict__ classes, const StepDesc *__restrict__ steps, const StepEnt *__restrict__ ents,
    const ClusterBlock *__restrict__ blocks, const PlanNet *__restrict__ pnets, const S *__restrict__ slices,
    double *__restrict__ w, int64_t n_slices, int64_t n_w, int n_ents, NetState *st) {
    using A = typename SliceIO<S>::acc;
    const ClusterBlock blk = blocks[xcd_block(blockIdx.x, gridDim.x)];
    const ClassDesc cd = classes[blk.cls];
    const int tid = threadIdx.x;
    bool bad = false;
    if constexpr (KIND >= 1 && KIND <= 4) {
        if (tid >= blk.count) return;
        const int f = blk.flat_begin + tid;
        const int net = f / cd.n_inst;
        const int k = f - net * cd.n_inst;
        const PlanNet pn = pnets[cd.pnet_begin + net];
        const InstStep *rec = cd.tab + (int64_t)k * cd.n_verts;
#ifdef PNE_CHECKED
        // every element the cycle reads: offsets xoff + a x0 + b x1, a, b < E
        for (int j = 0; j < cd.n_verts; ++j) {
            const int64_t lo = pn.slice_base + gld(&rec[j].xoff);
            const int64_t hi = lo + (int64_t)KIND * ((int64_t)gld(&rec[j].xs[0]) + gld(&rec[j].xs[1]));
            chk(lo, n_slices, bad);
            chk(hi, n_slices, bad);
        }
        const A v = bad ? A(0) : loop_trace<KIND + 1, S>(rec, cd.n_verts, slices, pn.slice_base);
#else
        const A v = loop_trace<KIND + 1, S>(rec, cd.n_verts, slices, pn.slice_base);
#endif
        w[chk(pn.w_base + gld(cd.iw + k), n_w, bad)] = (double)v;
        if (bad) atomicMin(&st[pn.net].status, PNE_ERR_CHECK);
        return;
    } else if constexpr (KIND == 5) {
        if (tid >= blk.count) return;
        const int f = blk.flat_begin + tid;
        const int net = f / cd.n_inst;
        const int k = f - net * cd.n_inst;
        const PlanNet pn = pnets[cd.pnet_begin + net];
        const InstStep *rec = cd.tab + (int64_t)k * cd.n_steps;
        A prod = A(1);
        for (int st2 = 0; st2 < cd.n_steps; ++st2)
            prod *= SliceIO<S>::load(slices, chk(pn.slice_base + gld(&rec[st2].xoff), n_slices, bad));
        w[chk(pn.w_base + gld(cd.iw + k), n_w, bad)] = (double)prod;
        if (bad) atomicMin(&st[pn.net].status, PNE_ERR_CHECK);
        return;
    } else {
        extern __shared__ double lds_raw[];
        __shared__ StepDesc s_steps[kMaxVerts];
        for (int i = tid; i < cd.n_steps * (int)(sizeof(StepDesc) / 4); i += kClThreads)
            reinterpret_cast<int32_t *>(s_steps)[i] =
                reinterpret_cast<const int32_t *>(steps + cd.step_begin)[i];
        const int g = cd.group;
        const int lane = tid & (g - 1);
        const int slot = tid / g;
        const bool valid = slot < blk.count;
        const int f = blk.flat_begin + (valid ? slot : 0);
        const int net = f / cd.n_inst;
        const int k = f - net * cd.n_inst;
        const PlanNet pn = pnets[cd.pnet_begin + net];
        const InstStep *rec = cd.tab + (int64_t)k * cd.n_steps;
        A *F = reinterpret_cast<A *>(lds_raw) + (size_t)slot * 2 * cd.max_f;
        A *G = F + cd.max_f;
        if (lane == 0) F[0] = A(1);
        __syncthreads();
        if (cd.max_sum > 0) {
            int2 *SO = reinterpret_cast<int2 *>(reinterpret_cast<A *>(lds_raw) + (size_t)(kClThreads / g) * 2 * cd.max_f) +
                       (size_t)slot * cd.max_sum;
            for (int st2 = 0; st2 < cd.n_steps; ++st2) {
                const StepDesc &sd = s_steps[st2];
                int xs[kMaxLab];
                int64_t xbase = 0;
                if (valid) {
                    // the record in three 16-byte loads (strides past n_xl are 0)
                    static_assert(sizeof(InstStep) == 48 && kMaxLab == 8, "InstStep layout");
                    const int4 *r4 = reinterpret_cast<const int4 *>(rec + st2);
                    const int4 ra = r4[0], rb = r4[1], rc = r4[2];
                    xbase = pn.slice_base + ra.x;
                    xs[0] = ra.y, xs[1] = ra.z, xs[2] = ra.w, xs[3] = rb.x;
                    xs[4] = rb.y, xs[5] = rb.z, xs[6] = rb.w, xs[7] = rc.x;
                    for (int t = lane; t < sd.n_sum; t += g) {
                        const StepEnt e = ents[chk(sd.ent + sd.n_out + t, n_ents, bad)];
                        SO[chk(t, cd.max_sum, bad)] = make_int2(e.f, ent_offset(e.xdig, xs));
                    }
                }
                wave_sync();
                if (valid) {
                    for (int o = lane; o < sd.n_out; o += g) {
                        const StepEnt e = ents[chk(sd.ent + o, n_ents, bad)];
                        const int64_t xb = xbase + ent_offset(e.xdig, xs);
                        // summed entries four, then two, then one at a time:
                        // a group's loads issue together, the products still
                        // accumulate in order
                        A acc = A(0);
                        int t = 0;
                        for (; t + 4 <= sd.n_sum; t += 4)
                            acc = sum_entries<4>(acc, SO + t, F, e.f, cd.max_f, slices, xb, n_slices, bad);
                        if (t + 2 <= sd.n_sum) {
                            acc = sum_entries<2>(acc, SO + t, F, e.f, cd.max_f, slices, xb, n_slices, bad);
                            t += 2;
                        }
                        if (t < sd.n_sum) acc = sum_entries<1>(acc, SO + t, F, e.f, cd.max_f, slices, xb, n_slices, bad);
                        G[chk(o, cd.max_f, bad)] = acc;
                    }
                }
                wave_sync();
                A *tmp = F;
                F = G;
                G = tmp;
            }
        } else {
            for (int st2 = 0; st2 < cd.n_steps; ++st2) {
                const StepDesc &sd = s_steps[st2];
                if (valid) {
                    const int64_t xbase = pn.slice_base + gld(&rec[st2].xoff);
                    int xs[kMaxLab];
#pragma unroll
                    for (int m = 0; m < kMaxLab; ++m) xs[m] = m < sd.n_xl ? gld(&rec[st2].xs[m]) : 0;
                    for (int o = lane; o < sd.n_out; o += g) {
                        int rem = o, fb = 0, xb = 0;
                        for (int kk = sd.n_ol - 1; kk >= 0; --kk) {
                            const int dd = sd.out_dim[kk];
                            const int dg = rem % dd;
                            rem /= dd;
                            fb += dg * sd.out_fs[kk];
                            const int xl = sd.out_xl[kk];
                            if (xl >= 0) {
#pragma unroll
                                for (int m = 0; m < kMaxLab; ++m)
                                    if (m == xl) xb += dg * xs[m];
                            }
                        }
                        int sfs[kMaxLab], sxs[kMaxLab], sdg[kMaxLab];
#pragma unroll
                        for (int kk = 0; kk < kMaxLab; ++kk) {
                            sdg[kk] = 0;
                            sfs[kk] = 0;
                            sxs[kk] = 0;
                            if (kk < sd.n_sl) {
                                sfs[kk] = sd.sum_fs[kk];
#pragma unroll
                                for (int m = 0; m < kMaxLab; ++m)
                                    if (m == sd.sum_xl[kk]) sxs[kk] = xs[m];
                            }
                        }
                        A acc = A(0);
                        int fo = fb;
                        int64_t xo = xbase + xb;
                        for (int t = 0; t < sd.n_sum; ++t) {
                            acc += F[chk(fo, cd.max_f, bad)] * SliceIO<S>::load(slices, chk(xo, n_slices, bad));
#pragma unroll
                            for (int kk = kMaxLab - 1; kk >= 0; --kk) {
                                if (kk >= sd.n_sl) continue;
                                if (++sdg[kk] < sd.sum_dim[kk]) {
                                    fo += sfs[kk];
                                    xo += sxs[kk];
                                    break;
                                }
                                fo -= (sd.sum_dim[kk] - 1) * sfs[kk];
                                xo -= (int64_t)(sd.sum_dim[kk] - 1) * sxs[kk];
                                sdg[kk] = 0;
                            }
                        }
                        G[chk(o, cd.max_f, bad)] = acc;
                    }
                }
                // an instance's lanes lie in one wavefront (g divides 64), and F and
                // G are its own: a wavefront-scope fence orders the step's LDS
                // writes before the next step's reads, and the waves of the block
                // run their steps independently
                wave_sync();
                A *t = F;
                F = G;
                G = t;
            }
        }
        if (valid) {
            const int64_t wo = pn.w_base + gld(cd.iw + k);
            for (int o = lane; o < cd.out_size; o += g) w[chk(wo + o, n_w, bad)] = (double)F[chk(o, cd.max_f, bad)];
            if (bad) atomicMin(&st[pn.net].status, PNE_ERR_CHECK);
        }
    }
}

// Block sum of one value per thread in a fixed order (deterministic).
__device__ double block_sum(double v, double *red) {
    const int tid = threadIdx.x;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < kCbThreads / 64; ++k) t += red[k];
    __syncthreads();
    return t;
}

// Per network: FP64 sum of the retained configurations.  Clusters come in
// contiguous (type, size) buckets; with W_s the bucket sums, configurations of
// one or two vertex-disjoint clusters with total degree <= K are
//   sum_s W_s + sum_{s<s'} W_s W_s' + sum_s (W_s^2 - sum w^2)/2 - overlaps,
// the overlaps being the explicitly listed pairs of clusters that share a
// site.  Open networks combine vacuum vectors and open-cluster tensors the
// same way, one tensor product per configuration.
template <typename S>
__global__ void __launch_bounds__(kCbThreads) k_combine(const int *__restrict__ combine_nets,
                                                        const CombineRec *__restrict__ recs,
                                                        const GeoRec *__restrict__ geos,
                                                        const Bucket *__restrict__ buckets,
                                                        const int *__restrict__ pair_a, const int *__restrict__ pair_b,
                                                        const PairCat *__restrict__ cats,
                                                        const int *__restrict__ coll_off,
                                                        const int *__restrict__ coll_cl,
                                                        const double *__restrict__ coll_coef,
                                                        const double *__restrict__ w,
                                                        const double *__restrict__ site_log,
                                                        const int *__restrict__ site_sign, const double *__restrict__ vac,
                                                        const NetState *__restrict__ st, NetResult *__restrict__ out,
                                                        double *__restrict__ open_out,
                                                        const SiteRec *__restrict__ sites,
                                                        const S *__restrict__ slices) {
    const int net = combine_nets[blockIdx.x];
    const CombineRec cr = recs[net];
    const GeoRec gr = geos[cr.geo];
    __shared__ double red[kCbThreads / 64];
    __shared__ double bsum[64][kMaxOpenOut];
    __shared__ double bsq[64];
    __shared__ double psum[8][kMaxOpenOut];
    __shared__ int bidx[4][33];
    const int tid = threadIdx.x;
    const double *wn = w + cr.w_base;

    double lg = 0.0, neg = 0.0;
    for (int s = tid; s < cr.n_sites; s += kCbThreads) {
        lg += site_log[cr.site_begin + s];
        neg += site_sign[cr.site_begin + s] < 0 ? 1.0 : 0.0;
    }
    lg = block_sum(lg, red);
    neg = block_sum(neg, red);
    double dangling, err;
    net_diagnostics<kCbThreads, S>(cr, gr, buckets, sites, slices, wn, red, &dangling, &err);

    if (gr.listed) {
        // User partitions (closed networks): every retained configuration is
        // listed with its clusters; its value is the product of their
        // weights, times its integer coefficient under recursive
        // partitioning.  Each thread sums its configurations in list order,
        // then the block sum adds the per-thread sums in a fixed order.
        const int *off = coll_off + gr.coll_begin;
        const int *cls = coll_cl + gr.coll_cl_begin;
        const double *coef = gr.coef_begin >= 0 ? coll_coef + gr.coef_begin : nullptr;
        double v = 0.0;
        for (int k = tid; k < gr.n_colls; k += kCbThreads) {
            double prod = coef ? gld(&coef[k]) : 1.0;
            const int j1 = gld(&off[k + 1]);
            for (int j = gld(&off[k]); j < j1; ++j) prod *= wn[gld(&cls[j])];
            v += prod;
        }
        v = block_sum(v, red);
        if (tid != 0) return;
        NetResult res;
        res.status = st[net].status;
        res.log_bp = lg;
        res.sum = v;
        res.dangling = dangling;
        const int sign_bp = ((int)neg & 1) ? -1 : 1;
        const double tot = 1.0 + v;
        res.err_est = err / fabs(tot);
        res.sign = tot == 0.0 ? 0 : (tot > 0.0 ? sign_bp : -sign_bp);
        res.log_abs = lg + log(fabs(tot));
        out[net] = res;
        return;
    }

    for (int i = tid; i < 4 * 33; i += kCbThreads) bidx[i / 33][i % 33] = -1;
    __syncthreads();
    const int nb = gr.n_buckets < 64 ? gr.n_buckets : 64;
    for (int b = 0; b < nb; ++b) {
        const Bucket bk = buckets[gr.bucket_begin + b];
        if (tid == 0 && bk.size <= 32) bidx[bk.type][bk.size] = b;
        for (int e = 0; e < bk.osz; ++e) {
            double v = 0.0;
            for (int c = bk.begin + tid; c < bk.end; c += kCbThreads) v += wn[bk.w_begin + (int64_t)(c - bk.begin) * bk.osz + e];
            v = block_sum(v, red);
            if (tid == 0) bsum[b][e] = v;
        }
        if (bk.type == 0) {
            double v = 0.0;
            for (int c = bk.begin + tid; c < bk.end; c += kCbThreads) {
                double x = wn[bk.w_begin + (c - bk.begin)];
                v = fma(x, x, v);
            }
            v = block_sum(v, red);
            if (tid == 0) bsq[b] = v;
        }
    }
    // overlap pair sums per category (index: 0 closed-closed, 1 A-closed,
    // 2 B-closed, 3 AB-closed, 4 B-with-A)
    const int pa = cr.pa, pb = cr.pb;
    for (int k = 0; k < 5; ++k)
        for (int e = tid; e < kMaxOpenOut; e += kCbThreads) psum[k][e] = 0.0;
    __syncthreads();
    for (int ci = 0; ci < gr.n_pair_cats; ++ci) {
        const PairCat pc = cats[gr.pair_cat_begin + ci];
        int slot, osz;
        if (pc.t2 == 0) {
            slot = pc.t1;
            osz = pc.t1 == 0 ? 1 : pc.t1 == 1 ? pa : pc.t1 == 2 ? pb : pa * pb;
        } else {
            slot = 4;
            osz = pa * pb;
        }
        // weight offsets: clusters within a type are contiguous, so locate by bucket
        for (int e = 0; e < osz; ++e) {
            double v = 0.0;
            for (int p = pc.begin + tid; p < pc.end; p += kCbThreads) {
                const int ca = pair_a[gr.pair_begin + p], cb = pair_b[gr.pair_begin + p];
                // offsets through the bucket tables (type-ordered clusters)
                int64_t oa = -1, ob = -1;
                int sa = 1, sb = 1;
                for (int b = 0; b < nb; ++b) {
                    const Bucket bk = buckets[gr.bucket_begin + b];
                    if (ca >= bk.begin && ca < bk.end) {
                        oa = bk.w_begin + (int64_t)(ca - bk.begin) * bk.osz;
                        sa = bk.osz;
                    }
                    if (cb >= bk.begin && cb < bk.end) {
                        ob = bk.w_begin + (int64_t)(cb - bk.begin) * bk.osz;
                        sb = bk.osz;
                    }
                }
                if (slot == 4) {
                    // B-cluster (ca) with A-cluster (cb): entry e = (ia, ib)
                    const int ia = e / pb, ib = e % pb;
                    v = fma(wn[ob + ia], wn[oa + ib], v);
                } else {
                    (void)sa;
                    (void)sb;
                    v = fma(wn[oa + e], wn[ob], v);
                }
            }
            v = block_sum(v, red);
            if (tid == 0) psum[slot][e] = v;
        }
    }
    __syncthreads();
    if (tid != 0) return;

    NetResult res;
    const NetState ns = st[net];
    res.status = ns.status;
    res.log_bp = lg;
    const int sign_bp = ((int)neg & 1) ? -1 : 1;
    const int K = gr.K < 32 ? gr.K : 32;
    auto B = [&](int t, int s) { return (s >= 0 && s <= 32) ? bidx[t][s] : -1; };
    double SC = 0.0;
    for (int s = 1; s <= K; ++s) {
        int b = B(0, s);
        if (b >= 0) SC += bsum[b][0];
    }
    for (int s = 1; s <= K; ++s) {
        int b = B(0, s);
        if (b < 0) continue;
        for (int s2 = s + 1; s + s2 <= K; ++s2) {
            int b2 = B(0, s2);
            if (b2 >= 0) SC += bsum[b][0] * bsum[b2][0];
        }
        if (2 * s <= K) SC += 0.5 * (bsum[b][0] * bsum[b][0] - bsq[b]);
    }
    SC -= psum[0][0];
    res.sum = SC;
    res.dangling = dangling;
    if (cr.cumulant) {
        double bw0[64], bq0[64];
        for (int b = 0; b < nb; ++b) {
            bw0[b] = bsum[b][0];
            bq0[b] = bsq[b];
        }
        res.sum = cumulant_form(bw0, bq0, [&](int s) { return B(0, s); }, K, psum[0][0]);
        res.sign = sign_bp;
        res.log_abs = lg + res.sum;
        res.err_est = err;
    } else if (cr.vac_a < 0) {
        const double tot = 1.0 + SC;
        res.sign = tot == 0.0 ? 0 : (tot > 0.0 ? sign_bp : -sign_bp);
        res.log_abs = lg + log(fabs(tot));
        res.err_est = err / fabs(tot);
    } else {
        // Wc(<= budget) helper: sum of closed bucket sums with size <= budget
        auto wc_upto = [&](int budget) {
            double v = 0.0;
            for (int s = 1; s <= budget && s <= K; ++s) {
                int b = B(0, s);
                if (b >= 0) v += bsum[b][0];
            }
            return v;
        };
        double xa[kMaxOpenOut], xb[kMaxOpenOut];
        for (int i = 0; i < pa; ++i) xa[i] = vac[cr.vac_a + i];
        for (int j = 0; j < pb; ++j) xb[j] = cr.vac_b >= 0 ? vac[cr.vac_b + j] : 1.0;
        double VA[kMaxOpenOut], VB[kMaxOpenOut];
        double omax = 0.0;
        for (int i = 0; i < pa; ++i) {
            double v = 0.0;
            for (int s = 1; s <= K; ++s) {
                int b = B(1, s);
                if (b >= 0) v += bsum[b][i] * (1.0 + wc_upto(K - s));
            }
            VA[i] = v - psum[1][i];
        }
        for (int j = 0; j < pb; ++j) {
            double v = 0.0;
            for (int s = 1; s <= K; ++s) {
                int b = B(2, s);
                if (b >= 0) v += bsum[b][j] * (1.0 + wc_upto(K - s));
            }
            VB[j] = v - psum[2][j];
        }
        for (int i = 0; i < pa; ++i)
            for (int j = 0; j < pb; ++j) {
                const int e = i * pb + j;
                double v = xa[i] * xb[j] * (1.0 + SC) + VA[i] * xb[j] + xa[i] * VB[j];
                for (int s = 1; s <= K; ++s) {
                    int b = B(3, s);
                    if (b >= 0) v += bsum[b][e] * (1.0 + wc_upto(K - s));
                }
                v -= psum[3][e];
                for (int s = 1; s <= K; ++s) {
                    int b = B(1, s);
                    if (b < 0) continue;
                    for (int s2 = 1; s + s2 <= K; ++s2) {
                        int b2 = B(2, s2);
                        if (b2 >= 0) v += bsum[b][i] * bsum[b2][j];
                    }
                }
                v -= psum[4][e];
                open_out[cr.open_off + e] = sign_bp * v;
                omax = fmax(omax, fabs(v));
            }
        res.sign = sign_bp;
        res.log_abs = lg;
        res.err_est = omax > 0.0 ? err / omax : err;
    }
    out[net] = res;
}

}  // namespace

int regauge_table_doubles(int dim, int rank) { return regauge_call_table(dim, rank); }

bool regauge_reg_supported(int dim, int rank) {
    if (dim < 2 || dim > 6 || rank < 1 || rank > 6) return false;
    const int B = dim <= 2 ? 1 : (dim <= 4 ? 2 : 3);
    const int T = (6 / B) < rank ? (6 / B) : rank;
    return rg_ipow(dim, rank - T) <= 4;
}

bool regauge_wide_supported(int dim, int rank) {
    switch (dim * 8 + rank) {
        case 3 * 8 + 5: case 4 * 8 + 5: case 5 * 8 + 3: case 6 * 8 + 3:
            return true;
        default:
            return false;
    }
}

int regauge_wide_sites(int dim, int rank) { return regauge_wide_supported(dim, rank) ? regauge_sites_per_tile(dim, rank) : 0; }

template <typename S>
static void launch_regauge_t(const DeviceBatch &b, hipStream_t s) {
    if (b.n_rg_tiles)
        hipLaunchKernelGGL(k_regauge_tiles<S>, dim3(b.n_rg_tiles), dim3(64), 0, s, b.all_tiles, b.rg_tiles, b.sites,
                           b.tile_sites, b.msg0, b.msg1, (S *)b.slices, b.site_log, b.site_sign, b.state);
    // the wide shapes, one launch per shape (rg_wide is grouped by shape)
    for (int g = 0; g < b.n_rg_wide_groups; ++g) {
        const int cnt = b.rg_wide_begin[g + 1] - b.rg_wide_begin[g];
        const int *idx = b.rg_wide + b.rg_wide_begin[g];
#define PNE_RGW(D_, R_)                                                                                       \
    case D_ * 8 + R_:                                                                                         \
        hipLaunchKernelGGL((k_regauge_wide<D_, R_, S>), dim3(cnt), dim3(64), 0, s, b.all_tiles, idx, b.sites,  \
                           b.tile_sites, b.msg0, b.msg1, (S *)b.slices, b.site_log, b.site_sign, b.state);      \
        break;
        switch (b.rg_wide_shape[g]) {
            PNE_RGW(3, 5) PNE_RGW(4, 5) PNE_RGW(5, 3) PNE_RGW(6, 3)
            default: break;
        }
#undef PNE_RGW
    }
    // one launch per size group: the dynamic LDS is twice the group's largest site
    for (int g = 0; g < b.n_rg_groups; ++g) {
        const int cnt = b.rg_group_begin[g + 1] - b.rg_group_begin[g];
        if (cnt > 0)
            hipLaunchKernelGGL(k_regauge<S>, dim3(cnt), dim3(kRgThreads), b.rg_group_lds[g], s, b.sites,
                               b.rg_sites + b.rg_group_begin[g], b.msg0, b.msg1, (S *)b.slices, b.site_log,
                               b.site_sign, b.vac, b.state);
    }
}

hipError_t launch_regauge(const DeviceBatch &b, hipStream_t s) {
    switch (b.precision) {
        case 0: launch_regauge_t<double>(b, s); break;
        case 1: launch_regauge_t<float>(b, s); break;
        default: launch_regauge_t<uint16_t>(b, s); break;
    }
    return hipGetLastError();
}

template <typename S, int KIND>
void launch_clusters_kind(const DeviceBatch &b, hipStream_t s) {
    const int b0 = b.cl_kind_begin[KIND], n = b.cl_kind_begin[KIND + 1] - b0;
    if (n > 0)
        hipLaunchKernelGGL((k_clusters<S, KIND>), dim3(n), dim3(kClThreads), KIND == 0 ? b.cluster_lds : 0, s,
                           b.classes, b.steps, b.step_ents, b.cblocks + b0, b.pnets, (const S *)b.slices, b.w,
                           b.n_slice_elems, b.n_w, b.n_step_ents, b.state);
}

template <typename S>
void launch_clusters_t(const DeviceBatch &b, hipStream_t s) {
    static_assert(DeviceBatch::kClKinds == 6, "cluster block kinds");
    launch_clusters_kind<S, 0>(b, s);
    launch_clusters_kind<S, 1>(b, s);
    launch_clusters_kind<S, 2>(b, s);
    launch_clusters_kind<S, 3>(b, s);
    launch_clusters_kind<S, 4>(b, s);
    launch_clusters_kind<S, 5>(b, s);
}

hipError_t launch_clusters(const DeviceBatch &b, hipStream_t s) {
    if (!b.n_cblocks) return hipSuccess;
    switch (b.precision) {
        case 0: launch_clusters_t<double>(b, s); break;
        case 1: launch_clusters_t<float>(b, s); break;
        default: launch_clusters_t<uint16_t>(b, s); break;
    }
    return hipGetLastError();
}

template <typename S>
static void launch_combine_t(const DeviceBatch &b, hipStream_t s) {
    hipLaunchKernelGGL(k_combine<S>, dim3(b.n_combine), dim3(kCbThreads), 0, s, b.combine_nets, b.crec, b.geos,
                       b.buckets, b.pair_a, b.pair_b, b.pair_cats, b.coll_off, b.coll_cl, b.coll_coef, b.w, b.site_log,
                       b.site_sign, b.vac, b.state, b.results, b.open_out, b.sites, (const S *)b.slices);
}

hipError_t launch_combine(const DeviceBatch &b, hipStream_t s) {
    if (!b.n_combine) return hipSuccess;
    switch (b.precision) {
        case 0: launch_combine_t<double>(b, s); break;
        case 1: launch_combine_t<float>(b, s); break;
        default: launch_combine_t<uint16_t>(b, s); break;
    }
    return hipGetLastError();
}

}  // namespace pne
