// Belief-propagation sweeps on gfx950 (Sec. II.B: the rank-1 projectors are
// built from fixed-point BP messages; Sec. III.D: an open leg's incoming
// message is its own outgoing message of the previous sweep).
//
//   k_init      uniform start messages 1/sqrt(d) and per-network state
//   k_bp_sweep  one Jacobi sweep; one wavefront per tile of same-shape sites;
//               each tile first applies the stop test to the previous sweep
//   k_bp_close  marks networks still running when the sweeps end
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dpp.h"
#include "gmem.h"
#include "kernels.h"

namespace pne {

namespace {

constexpr int kBpThreads = 64;  // one wavefront per tile

__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// floor(a / b) for 0 <= a < 2^22, 1 <= b <= 2^16, using b's reciprocal in
// FP32: (a + 0.5) / b stays within 0.5/b of the true quotient's floor + 0.5.
__device__ inline int fdiv(int a, float inv_b) { return (int)(((float)a + 0.5f) * inv_b); }

// State reset of the networks listed in init_nets and uniform initial
// messages 1/sqrt(d) for the sites listed in init_sites (networks swept launch
// by launch; a persistent block resets its network's state and initialises
// its messages in LDS itself).
__global__ void k_init(const SiteRec *__restrict__ sites, const int *__restrict__ init_sites, int n_sites,
                       double *__restrict__ msg0, NetState *__restrict__ st, const int *__restrict__ init_nets,
                       int n_nets) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_nets) {
        NetState s;
        s.stop = -1;
        s.iters = 0;
        s.parity = 0;
        s.status = 0;
        s.res_acc[0] = s.res_acc[1] = s.res_acc[2] = 0ull;
        s.best[0] = s.best[1] = INFINITY;
        s.best_at[0] = s.best_at[1] = -1;
        s.residual = 0.0;
        s.log_bp = 0.0;
        s.sign_bp = 1;
        s.converged = 0;
        s.t_start = s.t_bp = s.t_rg = 0ull;
        st[init_nets[i]] = s;
    }
    if (i < n_sites) {
        const SiteRec &r = sites[init_sites[i]];
        for (int l = 0; l < r.rank; ++l) {
            double v = 1.0 / sqrt((double)r.dim[l]);
            double *m = msg0 + r.msg_off + r.moff[l];
            for (int k = 0; k < r.dim[l]; ++k) m[k] = v;
        }
    }
}

// Stop test for sweep k of a network: true when the network stopped before
// sweep k.  Every tile of the network reaches the same answer, because it
// depends only on values completed by earlier launches (the residual of sweep
// k-1, the error status and the smallest-residual record in slot k&1).  The
// network's first tile records the stop, or else the record updated with
// sweep k-1 in the other slot.  A network also stops, as converged, at its
// rounding floor: no new smallest residual for `stall` sweeps, that residual
// at most `floor_tol`.
__device__ bool network_stopped(NetState *ns, int k, double tol, int max_iter, int stall, double floor_tol,
                                bool writer) {
    // every input is loaded, and every test evaluated, before the first
    // branch, so the loads share one round trip to memory; (k + 2) % 3 is
    // sweep k-1's residual slot, and an unused in-bounds slot at k = 0
    const int stop = ns->stop;
    const double r = __longlong_as_double((long long)ns->res_acc[(k + 2) % 3]);
    const int status = ns->status;
    const double best_in = ns->best[k & 1];
    const int best_at_in = ns->best_at[k & 1];
    const bool conv = status >= 0 && r <= tol;
    const bool better = !conv && r < best_in;
    const double best = better ? r : best_in;
    const int best_at = better ? k - 1 : best_at_in;
    const bool floor = !conv && !better && status >= 0 && stall > 0 && best_in <= floor_tol &&
                       (k - 1) - best_at_in >= stall;
    // the exits are combined without branches, so that no load is sunk
    // behind the first test
    const bool running = (stop < 0) & (k != 0);
    const bool end = (status < 0) | conv | floor | (k >= max_iter);
    if (writer & running) {
        if (end) {
            ns->stop = k - 1;
            ns->iters = k;
            ns->parity = k & 1;
            ns->residual = r;
            ns->converged = (conv || floor) ? 1 : 0;
        } else {
            ns->best[(k - 1) & 1] = best;
            ns->best_at[(k - 1) & 1] = best_at;
        }
    }
    return (stop >= 0) | (running & end);
}

// One tile of one sweep.  DC > 0: every leg has dimension DC (constant index
// arithmetic); DC == 0: per-leg dimensions from the tile's first site.
//
// The outgoing message on leg l is the site tensor contracted with the
// incoming messages of all other legs.  All of them come from peeling legs
// off the end: at the level of leg q the current tensor C over legs 0..q
// (C = T at the start) is viewed as rows (legs 0..q-1) of length d_q, and
//     next[row] = sum_i C[row, i] m_q[i]            (C with leg q contracted)
//     out_q[i]  = sum_row w(row) C[row, i],   w(row) = prod_{k<q} m_k[row_k];
// the last level leaves out_0 = C over leg 0.  Each out_q reduction is split
// over the lanes in two fixed-order stages (deterministic).
template <int N>
struct TileSharedN {
    const double *t[N];
    int msg[N];
    int dst[N * kMaxRank];
    int dim[kMaxRank], moff[kMaxRank];
    int bad;
};
using TileShared = TileSharedN<64>;
constexpr int kFusedTileSites = 16;  // largest register tile inside the fused kernel

template <int DC>
__device__ void sweep_tile(const BpTile &tl, const SiteRec *__restrict__ sites, const int *__restrict__ tile_sites,
                           const double *__restrict__ min, double *__restrict__ mout, NetState *ns, int sweep,
                           double *lds, TileShared &sh, double damp) {
    const double **s_t = sh.t;
    int *s_msg = sh.msg;
    int *s_dst = sh.dst;
    int *s_dim = sh.dim;
    int *s_moff = sh.moff;
    int &s_bad = sh.bad;
    const int tid = threadIdx.x;
    const int R = tl.rank, size = tl.size, nos = tl.n_os, nsit = tl.n_sites;
    for (int j = tid; j < nsit; j += kBpThreads) {
        const SiteRec &r = sites[tile_sites[tl.site_begin + j]];
        s_t[j] = r.t;
        s_msg[j] = r.msg_off;
        for (int l = 0; l < R; ++l) s_dst[j * kMaxRank + l] = r.dst[l];
        if (j == 0) {
            for (int l = 0; l < R; ++l) {
                s_dim[l] = r.dim[l];
                s_moff[l] = r.moff[l];
            }
            s_bad = 0;
        }
    }
    __syncthreads();
    auto dim = [&](int l) { return DC > 0 ? DC : s_dim[l]; };
    auto moff = [&](int l) { return DC > 0 ? DC * l : s_moff[l]; };
    const int rows0 = size / dim(R - 1);
    double *lm = lds;                  // incoming messages           nsit * nos
    double *lold = lm + nsit * nos;    // partners' previous messages nsit * nos
    double *lo = lold + nsit * nos;    // raw outgoing messages       nsit * nos
    double *part = lo + nsit * nos;    // tensor / weighted rows      nsit * size
    double *cur = part + nsit * size;  // peeled tensor               nsit * rows0
    double *nxt = cur + nsit * rows0;  // next peeled tensor          nsit * rows0
    double *red = nxt + nsit * rows0;  // reduction partials          >= 64
    const float inv_size = 1.0f / (float)size;
    const float inv_nos = 1.0f / (float)nos;
    // the tiles' tensors, eight loads per lane in flight at a time
    for (int e0 = tid; e0 < nsit * size; e0 += 8 * kBpThreads) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int eu = e0 + u * kBpThreads;
            const int e = eu < nsit * size ? eu : nsit * size - 1;  // clamped in bounds
            const int j = fdiv(e, inv_size);
            v[u] = dev::gld(s_t[j] + (e - j * size));
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * kBpThreads;
            if (e < nsit * size) part[e] = v[u];
        }
    }
    for (int e = tid; e < nsit * nos; e += kBpThreads) {
        const int j = fdiv(e, inv_nos);
        const int r = e - j * nos;
        int l = 0;
        while (l + 1 < R && r >= moff(l + 1)) ++l;
        lm[e] = min[s_msg[j] + r];
        lold[e] = min[s_dst[j * kMaxRank + l] + (r - moff(l))];
    }
    __syncthreads();

    if (R == 1) {
        for (int e = tid; e < nsit * nos; e += kBpThreads) lo[e] = part[e];
    } else {
        int cnt = size;  // entries per site of the current tensor
        for (int q = R - 1; q >= 1; --q) {
            const int dq = dim(q);
            const int rows = cnt / dq;
            const float inv_rows = 1.0f / (float)rows;
            const double *src_base = (q == R - 1) ? part : cur;
            const int src_stride = (q == R - 1) ? size : rows0;
            for (int o = tid; o < nsit * rows; o += kBpThreads) {
                const int j = fdiv(o, inv_rows);
                const int r = o - j * rows;
                const double *mj = lm + j * nos;
                double w = 1.0;
                int rem = r;
                for (int k = q - 1; k >= 0; --k) {
                    const int dk = dim(k);
                    const int dg = rem % dk;
                    rem /= dk;
                    w *= mj[moff(k) + dg];
                }
                const double *mq = mj + moff(q);
                const double *src = src_base + j * src_stride + r * dq;
                double *pr = part + j * size + r * dq;
                double a = 0.0;
                if (DC > 0) {
#pragma unroll
                    for (int i = 0; i < (DC > 0 ? DC : 1); ++i) {
                        const double v = src[i];
                        a = fma(v, mq[i], a);
                        pr[i] = w * v;
                    }
                } else {
                    for (int i = 0; i < dq; ++i) {
                        const double v = src[i];
                        a = fma(v, mq[i], a);
                        pr[i] = w * v;
                    }
                }
                nxt[j * rows0 + r] = a;
            }
            __syncthreads();
            // out_q[j][i] = sum_r part[j][r][i], split into nch row chunks
            const int nbins = nsit * dq;
            const int nch = nbins >= kBpThreads ? 1 : (kBpThreads / nbins < rows ? kBpThreads / nbins : rows);
            const int chunk = (rows + nch - 1) / nch;
            const float inv_nbins = 1.0f / (float)nbins;
            for (int o = tid; o < nbins * nch; o += kBpThreads) {
                const int c = fdiv(o, inv_nbins);
                const int b = o - c * nbins;
                const int j = b / dq;
                const int i = b - j * dq;
                const double *pr = part + j * size + i;
                const int r1 = (c + 1) * chunk < rows ? (c + 1) * chunk : rows;
                double s = 0.0;
                for (int r = c * chunk; r < r1; ++r) s += pr[r * dq];
                red[o] = s;
            }
            __syncthreads();
            for (int b = tid; b < nbins; b += kBpThreads) {
                const int j = b / dq;
                const int i = b - j * dq;
                double s = 0.0;
                for (int c = 0; c < nch; ++c) s += red[c * nbins + b];
                lo[j * nos + moff(q) + i] = s;
            }
            double *t = cur;
            cur = nxt;
            nxt = t;
            cnt = rows;
            __syncthreads();
        }
        const int d0 = dim(0);
        for (int o = tid; o < nsit * d0; o += kBpThreads) {
            const int j = o / d0;
            const int i = o - j * d0;
            lo[j * nos + i] = cur[j * rows0 + i];
        }
    }
    __syncthreads();

    // normalise, write to the partner slots, residual
    double res = 0.0;
    for (int m = tid; m < nsit * R; m += kBpThreads) {
        const int j = m / R;
        const int l = m - j * R;
        const double *raw = lo + j * nos + moff(l);
        const double *old = lold + j * nos + moff(l);
        const int d = dim(l);
        double n2 = 0.0, sum = 0.0;
        for (int k = 0; k < d; ++k) {
            n2 = fma(raw[k], raw[k], n2);
            sum += raw[k];
        }
        const double nrm = sqrt(n2);
        if (!(nrm > 0.0) || !isfinite(nrm)) {
            s_bad = 1;
            continue;
        }
        const double inv = (sum < 0.0 ? -1.0 : 1.0) / nrm;  // L2 norm, sign fixed so the sum is >= 0
        double dinv = 1.0;  // damped: the mix is normalised and sign-fixed again
        if (damp > 0.0) {
            double m2 = 0.0, msum = 0.0;
            for (int k = 0; k < d; ++k) {
                const double x = (1.0 - damp) * (raw[k] * inv) + damp * old[k];
                m2 = fma(x, x, m2);
                msum += x;
            }
            const double mn = sqrt(m2);
            if (!(mn > 0.0) || !isfinite(mn)) {
                s_bad = 1;
                continue;
            }
            dinv = (msum < 0.0 ? -1.0 : 1.0) / mn;
        }
        const int dst = s_dst[j * kMaxRank + l];
        double d1 = 0.0, d2 = 0.0;
        for (int k = 0; k < d; ++k) {
            double v = raw[k] * inv;
            if (damp > 0.0) v = ((1.0 - damp) * v + damp * old[k]) * dinv;
            d1 = fmax(d1, fabs(v - old[k]));
            d2 = fmax(d2, fabs(v + old[k]));
            mout[dst + k] = v;
        }
        res = fmax(res, fmin(d1, d2));
    }
    res = wave_max(res);
    __syncthreads();
    if (tid == 0) {
        atomicMax(&ns->res_acc[sweep % 3], (unsigned long long)__double_as_longlong(res));
        if (s_bad) atomicMin(&ns->status, -4);
    }
}

// ---------------------------------------------------------------------------
// Register path for sites whose legs all have dimension D (R legs).  With
// P = D rounded up to a power of two, the last T legs (P^T <= 64) index lanes
// through bit-fields (digits >= D leave a lane idle); the first R-T legs
// ("lead" legs) index NL = D^(R-T) values each lane keeps in registers.
// SPW = 64 / P^T sites sit side by side in the wavefront and NS such rows are
// processed per tile, with every global load of the tile issued up front.
// Every outgoing message is a sum over lanes, done with xor butterflies
// inside the site's lane segment:
//   trailing leg m:  A * prod_{m' != m} m_{m'}[digit]  reduced over the other
//                    trailing bit-fields, A = sum_L T[L, lane] w(L) with the
//                    lead messages' product w(L);
//   lead leg k:      sum_{L: L_k = i} T[L, lane] prod_{k' != k} m_{k'}[L_{k'}]
//                    times the trailing messages, reduced over the segment.
template <int D>
struct RegShape {
    static constexpr int P = D <= 2 ? 2 : (D <= 4 ? 4 : 8);
    static constexpr int B = P == 2 ? 1 : (P == 4 ? 2 : 3);
};

constexpr int ipow(int b, int e) { return e <= 0 ? 1 : b * ipow(b, e - 1); }

__host__ __device__ constexpr int reg_trailing(int D, int R) {
    return (6 / (D <= 2 ? 1 : (D <= 4 ? 2 : 3))) < R ? (6 / (D <= 2 ? 1 : (D <= 4 ? 2 : 3))) : R;
}
__host__ __device__ constexpr int reg_rows(int D, int R) {
    return 1;
}

// Synchronisation inside one tile: the whole block (one wavefront per block)
// or only the wavefront (tiles processed by single waves of a larger block).
template <bool WAVE>
__device__ inline void tile_sync() {
    if (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    } else {
        __syncthreads();
    }
}

// Sum over trailing digit m2 of a register tile's lane field (B lane bits
// per digit, the last digit in the lowest bits).
template <int B, int T>
__device__ inline double trailing_digit_sum(double v, int m2) {
    if (m2 == T - 1) return dpp::bits_sum<0, B>(v);
    if constexpr (T >= 2)
        if (m2 == T - 2) return dpp::bits_sum<B, B>(v);
    if constexpr (T >= 3)
        if (m2 == T - 3) return dpp::bits_sum<2 * B, B>(v);
#pragma unroll
    for (int bit = 0; bit < B; ++bit) v += __shfl_xor(v, 1 << (B * (T - 1 - m2) + bit), 64);
    return v;
}

// Processes one register-path tile.  Message offsets in the site table are
// absolute; `min`/`mout` point at message storage for offset `msg_base`
// (global buffers with msg_base = 0, or a network's LDS copy).  Returns the
// tile's residual (valid in every lane); sets *bad on a zero message.
template <int D, int R, bool WAVE, class SH, int ROWS = 0>
__device__ double sweep_reg(const BpTile &tl, const SiteRec *__restrict__ sites, const int *__restrict__ tile_sites,
                            int my_site, const double *min, double *mout, int msg_base, double *lds, SH &sh,
                            int *bad, double damp) {
    constexpr int P = RegShape<D>::P;
    constexpr int B = RegShape<D>::B;
    constexpr int T = reg_trailing(D, R);
    constexpr int NLEG = R - T;
    constexpr int LS = 1 << (B * T);
    constexpr int SPW = 64 / LS;
    constexpr int NL = ipow(D, NLEG);
    constexpr int DT = ipow(D, T);
    constexpr int NS = ROWS > 0 ? ROWS : reg_rows(D, R);
    const int lane = threadIdx.x & 63;
    const int nsit = tl.n_sites;
    for (int j = lane; j < nsit; j += kBpThreads) {
        const SiteRec &r = sites[j == lane ? my_site : tile_sites[tl.site_begin + j]];
        sh.t[j] = r.t;
        sh.msg[j] = r.msg_off - msg_base;
#pragma unroll
        for (int l = 0; l < R; ++l) sh.dst[j * kMaxRank + l] = r.dst[l] - msg_base;
    }
    tile_sync<WAVE>();
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
    // every load of the tile up front
    double tv[NS][NL];
    double mt[NS][T];
    double ml[NS][NLEG > 0 ? NLEG : 1][D];
    bool act[NS];
#pragma unroll
    for (int row = 0; row < NS; ++row) {
        const int site = row * SPW + slot;
        act[row] = inseg && site < nsit;
        const int s = site < nsit ? site : 0;
        const double *tp = sh.t[s];
        const double *mi = min + sh.msg[s];
#pragma unroll
        for (int L = 0; L < NL; ++L) {
            const double x = dev::gld(tp + L * DT + toff);  // in bounds on every lane
            tv[row][L] = act[row] ? x : 0.0;
        }
#pragma unroll
        for (int m = 0; m < T; ++m) mt[row][m] = mi[(NLEG + m) * D + dig[m] % D];
#pragma unroll
        for (int k = 0; k < NLEG; ++k)
#pragma unroll
            for (int i = 0; i < D; ++i) ml[row][k][i] = mi[k * D + i];
    }
    const int nnorm = nsit * R;
    double oldv[D];
    if (lane < nnorm) {
        const int j = lane / R;
        const int l = lane - j * R;
        const int dst = sh.dst[j * kMaxRank + l];
#pragma unroll
        for (int k = 0; k < D; ++k) oldv[k] = min[dst + k];
    }

    double *out = lds;  // [site][R*D] raw outgoing messages
#pragma unroll
    for (int row = 0; row < NS; ++row) {
        const int site = row * SPW + slot;
        // lead-contracted value (more than 16 values per lane: four
        // interleaved partial sums, so the FMA chain is a quarter as long)
        constexpr int NA = NL > 16 ? 4 : 1;
        double Ap[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) Ap[a] = 0.0;
#pragma unroll
        for (int L = 0; L < NL; ++L) {
            double w = 1.0;
#pragma unroll
            for (int k = 0; k < NLEG; ++k) w *= ml[row][k][(L / ipow(D, NLEG - 1 - k)) % D];
            Ap[L % NA] = fma(tv[row][L], w, Ap[L % NA]);
        }
        double A = Ap[0];
#pragma unroll
        for (int a = 1; a < NA; ++a) A += Ap[a];
        // trailing legs
#pragma unroll
        for (int m = 0; m < T; ++m) {
            double pm = A;
#pragma unroll
            for (int m2 = 0; m2 < T; ++m2)
                if (m2 != m) pm *= mt[row][m2];
#pragma unroll
            for (int m2 = 0; m2 < T; ++m2) {
                if (m2 == m) continue;
                pm = trailing_digit_sum<B, T>(pm, m2);
            }
            bool owner = act[row];
#pragma unroll
            for (int m2 = 0; m2 < T; ++m2)
                if (m2 != m) owner = owner && dig[m2] == 0;
            if (owner) out[site * (R * D) + (NLEG + m) * D + dig[m]] = pm;
        }
        // lead legs
        if constexpr (NLEG > 0 && B * T == 6 && NLEG * D <= 16 && NL <= 36) {
            // one site per wavefront: the NLEG * D sums over all 64 lanes
            // at once, by recursive halving (lane i of the first row ends
            // with output i = k * D + j of lead leg k)
            double q = act[row] ? 1.0 : 0.0;
#pragma unroll
            for (int m = 0; m < T; ++m) q *= mt[row][m];
            auto lead = [&](int o) {
                const int k = o / D, i = o % D;
                double acc = 0.0;
#pragma unroll
                for (int L = 0; L < NL; ++L) {
                    if ((L / ipow(D, NLEG - 1 - k)) % D != i) continue;
                    double w = 1.0;
#pragma unroll
                    for (int k2 = 0; k2 < NLEG; ++k2)
                        if (k2 != k) w *= ml[row][k2][(L / ipow(D, NLEG - 1 - k2)) % D];
                    acc = fma(tv[row][L], w, acc);
                }
                return acc * q;
            };
            double sv[NLEG * D];
#pragma unroll
            for (int o = 0; o < NLEG * D; ++o) sv[o] = lead(o);
            const double tot = dpp::wave_sums16<NLEG * D>(sv, lane);
            if (lane < NLEG * D && site < nsit) out[site * (R * D) + lane] = tot;
        } else if (NLEG > 0) {
            double q = act[row] ? 1.0 : 0.0;
#pragma unroll
            for (int m = 0; m < T; ++m) q *= mt[row][m];
#pragma unroll
            for (int k = 0; k < NLEG; ++k) {
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    double sv = 0.0;
#pragma unroll
                    for (int L = 0; L < NL; ++L) {
                        if ((L / ipow(D, NLEG - 1 - k)) % D != i) continue;
                        double w = 1.0;
#pragma unroll
                        for (int k2 = 0; k2 < NLEG; ++k2)
                            if (k2 != k) w *= ml[row][k2][(L / ipow(D, NLEG - 1 - k2)) % D];
                        sv = fma(tv[row][L], w, sv);
                    }
                    sv *= q;
                    if constexpr (B * T == 6) {
                        sv = dpp::wave_sum(sv);  // every lane bit: the row by DPP, then the rows
                    } else {
#pragma unroll
                        for (int bit = 0; bit < B * T; ++bit) sv += __shfl_xor(sv, 1 << bit, 64);
                    }
                    if (tb == 0 && site < nsit) out[site * (R * D) + k * D + i] = sv;
                }
            }
        }
    }
    tile_sync<WAVE>();
    // normalise, write to the partner slots, residual
    double res = 0.0;
    for (int n = lane; n < nnorm; n += kBpThreads) {
        const int j = n / R;
        const int l = n - j * R;
        if (n != lane) {
            const int dst = sh.dst[j * kMaxRank + l];
#pragma unroll
            for (int k = 0; k < D; ++k) oldv[k] = min[dst + k];
        }
        const double *raw = out + j * (R * D) + l * D;
        double n2 = 0.0, sum = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            n2 = fma(raw[k], raw[k], n2);
            sum += raw[k];
        }
        const double nrm = sqrt(n2);
        if (!(nrm > 0.0) || !isfinite(nrm)) {
            *bad = 1;
            continue;
        }
        const double inv = (sum < 0.0 ? -1.0 : 1.0) / nrm;  // L2 norm, sign fixed so the sum is >= 0
        double dinv = 1.0;  // damped: the mix is normalised and sign-fixed again
        if (damp > 0.0) {
            double m2 = 0.0, msum = 0.0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double x = (1.0 - damp) * (raw[k] * inv) + damp * oldv[k];
                m2 = fma(x, x, m2);
                msum += x;
            }
            const double mn = sqrt(m2);
            if (!(mn > 0.0) || !isfinite(mn)) {
                *bad = 1;
                continue;
            }
            dinv = (msum < 0.0 ? -1.0 : 1.0) / mn;
        }
        const int dst = sh.dst[j * kMaxRank + l];
        double d1 = 0.0, d2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double v = raw[k] * inv;
            if (damp > 0.0) v = ((1.0 - damp) * v + damp * oldv[k]) * dinv;
            d1 = fmax(d1, fabs(v - oldv[k]));
            d2 = fmax(d2, fabs(v + oldv[k]));
            mout[dst + k] = v;
        }
        res = fmax(res, fmin(d1, d2));
    }
    res = wave_max(res);
    tile_sync<WAVE>();
    return res;
}

// Sites per register-path tile for (D, R) with at most `max_lead` values per
// lane, or 0 when the shape takes the LDS path.
__host__ __device__ constexpr int reg_sites_per_tile(int D, int R, int max_lead = 16) {
    return (D < 2 || D > 6 || R < 1 || R > 6 || ipow(D, R - reg_trailing(D, R)) > max_lead)
               ? 0
               : reg_rows(D, R) * (64 >> ((D <= 2 ? 1 : (D <= 4 ? 2 : 3)) * reg_trailing(D, R)));
}
// The per-launch sweep also keeps rank-4 sites of D = 5 and 6 and rank-6
// sites of D = 3 in registers (25, 36 and 27 values per lane, one site per
// wavefront): the wide shapes, swept by their own kernel.
__host__ __device__ constexpr bool wide_shape(int D, int R) {
    return (R == 4 && (D == 5 || D == 6)) || (R == 6 && D == 3);
}
// Rank-6 sites at D = 4 (the interior of 3D lattices, 4096 entries): three
// legs index the 64 lanes and the other three 64 values per lane, one site
// per wavefront, in a kernel instance of their own (its registers would hold
// every other tile to one wavefront per SIMD).
__host__ __device__ constexpr bool xwide_shape(int D, int R) { return R == 6 && D == 4; }

// One Jacobi sweep: sweep reads message buffer sweep&1 and writes the other.
// Tiles of networks that stopped exit at once; the per-network bookkeeping of
// the previous sweep is folded into the stop test, so one launch is one sweep
// and no block waits for, or fences against, any other block.
//
// WIDE: 0 the register and LDS tiles; 1 the register tiles of the wide
// shapes (wide_shape), 2 those of the extra-wide shape (xwide_shape), each
// kept apart so that their registers do not lower the occupancy of the
// other tiles.
template <int WIDE>
__global__ void __launch_bounds__(kBpThreads) __attribute__((amdgpu_waves_per_eu(WIDE == 1 ? 4 : 1)))
k_bp_sweep(const SiteRec *__restrict__ sites,
                                                         const BpTile *__restrict__ tiles,
                                                         const int *__restrict__ tile_sites,
                                                         double *msg0, double *msg1, NetState *st, int sweep,
                                                         double tol, int max_iter, int stall,
                                                         double floor_tol, double damp) {
    const BpTile tl = tiles[blockIdx.x];
    NetState *ns = st + tl.net;
    extern __shared__ double lds[];
    __shared__ int s_skip;
    __shared__ TileShared sh;
    // this lane's site of a register tile (clamped in bounds), loaded beside
    // the stop test's inputs rather than after them
    const int my_site = tile_sites[tl.site_begin + min((int)threadIdx.x, tl.n_sites - 1)];
    if (threadIdx.x == 0) {
        s_skip = network_stopped(ns, sweep, tol, max_iter, stall, floor_tol, tl.first != 0);
        // slot (sweep+1)%3 was last read at the start of sweep-1: clear it for sweep+1
        if (!s_skip && tl.first) ns->res_acc[(sweep + 1) % 3] = 0ull;
    }
    __syncthreads();
    if (s_skip) return;
    const double *min = (sweep & 1) ? msg1 : msg0;
    double *mout = (sweep & 1) ? msg0 : msg1;
    if constexpr (WIDE != 0) {
        if (threadIdx.x == 0) sh.bad = 0;
        double res = 0.0;
        if constexpr (WIDE == 2) {
            if (tl.dc == 4 && tl.rank == 6)
                res = sweep_reg<4, 6, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp);
            else
                sh.bad = 1;  // not the extra-wide shape: never scheduled here
        } else {
            switch (tl.dc * 8 + tl.rank) {
                case 30: res = sweep_reg<3, 6, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
                case 44: res = sweep_reg<5, 4, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
                case 52: res = sweep_reg<6, 4, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
                default: sh.bad = 1; break;  // not a wide shape: never scheduled here
            }
        }
        if (threadIdx.x == 0) {
            atomicMax(&ns->res_acc[sweep % 3], (unsigned long long)__double_as_longlong(res));
            if (sh.bad) atomicMin(&ns->status, -4);
        }
        return;
    }
    if (tl.reg) {
        double res = -1.0;
        if (threadIdx.x == 0) sh.bad = 0;
        switch (tl.dc * 8 + tl.rank) {
            case 17: res = sweep_reg<2, 1, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 18: res = sweep_reg<2, 2, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 19: res = sweep_reg<2, 3, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 20: res = sweep_reg<2, 4, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 21: res = sweep_reg<2, 5, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 22: res = sweep_reg<2, 6, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 25: res = sweep_reg<3, 1, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 26: res = sweep_reg<3, 2, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 27: res = sweep_reg<3, 3, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 28: res = sweep_reg<3, 4, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 29: res = sweep_reg<3, 5, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 33: res = sweep_reg<4, 1, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 34: res = sweep_reg<4, 2, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 35: res = sweep_reg<4, 3, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 36: res = sweep_reg<4, 4, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 37: res = sweep_reg<4, 5, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 41: res = sweep_reg<5, 1, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 42: res = sweep_reg<5, 2, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 43: res = sweep_reg<5, 3, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 49: res = sweep_reg<6, 1, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 50: res = sweep_reg<6, 2, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            case 51: res = sweep_reg<6, 3, false>(tl, sites, tile_sites, my_site, min, mout, 0, lds, sh, &sh.bad, damp); break;
            default: break;
        }
        if (res >= 0.0) {
            if (threadIdx.x == 0) {
                atomicMax(&ns->res_acc[sweep % 3], (unsigned long long)__double_as_longlong(res));
                if (sh.bad) atomicMin(&ns->status, -4);
            }
            return;
        }
    }
    switch (tl.dc) {
        case 2: sweep_tile<2>(tl, sites, tile_sites, min, mout, ns, sweep, lds, sh, damp); break;
        case 3: sweep_tile<3>(tl, sites, tile_sites, min, mout, ns, sweep, lds, sh, damp); break;
        case 4: sweep_tile<4>(tl, sites, tile_sites, min, mout, ns, sweep, lds, sh, damp); break;
        case 5: sweep_tile<5>(tl, sites, tile_sites, min, mout, ns, sweep, lds, sh, damp); break;
        case 6: sweep_tile<6>(tl, sites, tile_sites, min, mout, ns, sweep, lds, sh, damp); break;
        default: sweep_tile<0>(tl, sites, tile_sites, min, mout, ns, sweep, lds, sh, damp); break;
    }
}


// After the last launched sweep k_last: record networks that are still running.
__global__ void k_bp_close(NetState *st, int n_nets, int k_last, double tol) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_nets) return;
    NetState *ns = st + i;
    if (ns->stop >= 0) return;
    const double r = __longlong_as_double((long long)ns->res_acc[k_last % 3]);
    ns->stop = k_last;
    ns->iters = k_last + 1;
    ns->parity = (k_last + 1) & 1;
    ns->residual = r;
    ns->converged = (ns->status >= 0 && r <= tol) ? 1 : 0;
}

}  // namespace

int bp_tile_threads() { return kBpThreads; }

int bp_reg_sites_per_tile(int D, int R) { return reg_sites_per_tile(D, R); }
int bp_sweep_reg_sites_per_tile(int D, int R) {
    if (xwide_shape(D, R)) return reg_sites_per_tile(D, R, 64);
    return wide_shape(D, R) ? reg_sites_per_tile(D, R, 36) : reg_sites_per_tile(D, R);
}
bool bp_sweep_xwide(int D, int R) { return xwide_shape(D, R); }

size_t bp_tile_lds_doubles(int n_sites, int size, int n_os, int last_dim, int max_dim) {
    size_t red = (size_t)n_sites * (size_t)max_dim;
    if (red < (size_t)kBpThreads) red = kBpThreads;
    return (size_t)n_sites * (3 * (size_t)n_os + (size_t)size + 2 * (size_t)(size / last_dim)) + red;
}

hipError_t launch_init(const DeviceBatch &b, hipStream_t s) {
    int n = b.n_init_sites > b.n_init_nets ? b.n_init_sites : b.n_init_nets;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_init, dim3((n + 255) / 256), dim3(256), 0, s, b.sites, b.init_sites, b.n_init_sites,
                       b.msg0, b.state, b.init_nets, b.n_init_nets);
    return hipGetLastError();
}

// Three launches, each with the dynamic LDS its tiles need: a network's LDS
// tiles (tens of KB for large mixed-dimension sites) would otherwise hold
// every register tile of the sweep to a few blocks per CU.  Where the batch
// has a side stream and wide tiles, the register and LDS tiles of the other
// shapes run on the side stream, beside the wide launch.
hipError_t launch_sweep(const DeviceBatch &b, int k, double tol, int max_iter, hipStream_t s) {
    const int n_wide = b.n_wide_end - b.n_narrow_tiles;
    const int n_xwide = b.n_tiles - b.n_wide_end;
    const bool split = b.side != nullptr && n_wide + n_xwide > 0 && b.n_narrow_tiles > 0;
    hipError_t e = hipSuccess;
    hipStream_t ns = s;
    if (split) {
        if ((e = hipEventRecord(b.fork, s)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(b.side, b.fork, 0)) != hipSuccess) return e;
        ns = b.side;
    }
    if (b.n_reg_tiles > 0)
        hipLaunchKernelGGL(k_bp_sweep<0>, dim3(b.n_reg_tiles), dim3(kBpThreads), b.reg_lds, ns, b.sites, b.tiles,
                           b.tile_sites, b.msg0, b.msg1, b.state, k, tol, max_iter, b.bp_stall, b.bp_floor, b.damping);
    if (b.n_narrow_tiles > b.n_reg_tiles)
        hipLaunchKernelGGL(k_bp_sweep<0>, dim3(b.n_narrow_tiles - b.n_reg_tiles), dim3(kBpThreads), b.bp_lds, ns,
                           b.sites, b.tiles + b.n_reg_tiles, b.tile_sites, b.msg0, b.msg1, b.state, k, tol, max_iter,
                           b.bp_stall, b.bp_floor, b.damping);
    if (n_wide > 0)
        hipLaunchKernelGGL(k_bp_sweep<1>, dim3(n_wide), dim3(kBpThreads), b.wide_lds, s, b.sites,
                           b.tiles + b.n_narrow_tiles, b.tile_sites, b.msg0, b.msg1, b.state, k, tol, max_iter,
                           b.bp_stall, b.bp_floor, b.damping);
    if (n_xwide > 0)
        hipLaunchKernelGGL(k_bp_sweep<2>, dim3(n_xwide), dim3(kBpThreads), b.xwide_lds, s, b.sites,
                           b.tiles + b.n_wide_end, b.tile_sites, b.msg0, b.msg1, b.state, k, tol, max_iter,
                           b.bp_stall, b.bp_floor, b.damping);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (split) {
        if ((e = hipEventRecord(b.join, b.side)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, b.join, 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_close(const DeviceBatch &b, int k_last, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_bp_close, dim3((b.n_nets + 255) / 256), dim3(256), 0, s, b.state, b.n_nets, k_last, tol);
    return hipGetLastError();
}

}  // namespace pne
