// Rank-r projectors from weight passing (Sec. V, Appendix C) on small closed
// lattice networks, batched: one block per network runs the weight-passing
// sweeps (Eqs. (C1)-(C3)) with one-sided Jacobi SVDs, then one block
// per (network, term) contracts the gauged lattice with a diagonal operator
// on every bond (the weight S_b restricted to its first r indices for P, to
// the rest for Q, or whole), and one block per network adds the terms of the
// linear (Eq. (4)) or combinatorial (Eq. (7)) form.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dpp.h"
#include "gmem.h"
#include "pne.h"
#include "rankr.h"
#include "runtime.h"

namespace pne {
namespace {

using dev::gld;

constexpr int kRkChi = 4;        // bond dimension of the small-chi kernels
constexpr int kRkSite = kRkChi * kRkChi * kRkChi * kRkChi;  // entries of one site tensor
constexpr int kRkState = 1024;   // entries of the row-contraction state
constexpr int kRkWp = 64;        // threads of the weight-passing block

__device__ inline int tsize(int rank, int chi) {
    int n = 1;
    for (int l = 0; l < rank; ++l) n *= chi;
    return n;
}

// One-sided Jacobi SVD of the m x n matrix held column-major in a (column j
// at a[j * m ..]), n <= 4, by one wave of 64 lanes (at n = 4 two disjoint
// column pairs rotate at once, one per half-wave).  On return the columns
// are U S (orthogonal, norms s), V holds the accumulated rotations (n x n,
// V[i * n + j]), and s the column norms; columns, s and V are sorted by
// decreasing s.  Rotations stop when every pair is orthogonal to 1e-15
// relative, or after 60 sweeps.
__device__ void jacobi_svd(double *a, int m, int n, double *V, double *s) {
    const int lane = threadIdx.x;
    if (lane < n * n) V[lane] = (lane / n == lane % n) ? 1.0 : 0.0;
    __syncthreads();
    for (int sweep = 0; sweep < 60; ++sweep) {
        int rotated = 0;
        if (n == 4) {
            // the six pairs in three rounds of two disjoint pairs, one pair
            // per half-wave: (0,1)(2,3), (0,2)(1,3), (0,3)(1,2)
            const int half = lane >> 5, hl = lane & 31;
            for (int round = 0; round < 3; ++round) {
                const int p = half == 0 ? 0 : (round == 0 ? 2 : 1);
                const int q = half == 0 ? round + 1 : (round == 2 ? 2 : 3);
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = hl; i < m; i += 32) {
                    const double x = a[p * m + i], y = a[q * m + i];
                    al = fma(x, x, al);
                    be = fma(y, y, be);
                    ga = fma(x, y, ga);
                }
                // a 16-lane row butterfly on the VALU (DPP), then across the
                // half-wave's two rows
                al = dpp::row_sum(al);
                be = dpp::row_sum(be);
                ga = dpp::row_sum(ga);
                al += __shfl_xor(al, 16, 64);
                be += __shfl_xor(be, 16, 64);
                ga += __shfl_xor(ga, 16, 64);
                // the half's first lane's sums for all its lanes (see below)
                al = __shfl(al, half << 5, 64);
                be = __shfl(be, half << 5, 64);
                ga = __shfl(ga, half << 5, 64);
                if (!(fabs(ga) <= 1e-15 * sqrt(al * be) || ga == 0.0)) {
                    rotated = 1;
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                    for (int i = hl; i < m; i += 32) {
                        const double x = a[p * m + i], y = a[q * m + i];
                        a[p * m + i] = c * x - sn * y;
                        a[q * m + i] = sn * x + c * y;
                    }
                    if (hl < n) {
                        const double x = V[hl * n + p], y = V[hl * n + q];
                        V[hl * n + p] = c * x - sn * y;
                        V[hl * n + q] = sn * x + c * y;
                    }
                }
                __syncthreads();
            }
            if (!__any(rotated)) break;
            continue;
        }
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = lane; i < m; i += kRkWp) {
                    const double x = a[p * m + i], y = a[q * m + i];
                    al = fma(x, x, al);
                    be = fma(y, y, be);
                    ga = fma(x, y, ga);
                }
                al = dpp::wave_sum(al);
                be = dpp::wave_sum(be);
                ga = dpp::wave_sum(ga);
                // one lane's sums for the whole wave: the butterfly's can differ
                // in the last bit between lanes, enough to flip the rotation's
                // sign on tied column norms
                al = __shfl(al, 0, 64);
                be = __shfl(be, 0, 64);
                ga = __shfl(ga, 0, 64);
                if (fabs(ga) <= 1e-15 * sqrt(al * be) || ga == 0.0) continue;
                rotated = 1;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                for (int i = lane; i < m; i += kRkWp) {
                    const double x = a[p * m + i], y = a[q * m + i];
                    a[p * m + i] = c * x - sn * y;
                    a[q * m + i] = sn * x + c * y;
                }
                if (lane < n) {
                    const double x = V[lane * n + p], y = V[lane * n + q];
                    V[lane * n + p] = c * x - sn * y;
                    V[lane * n + q] = sn * x + c * y;
                }
                __syncthreads();
            }
        if (!rotated) break;
    }
    for (int j = 0; j < n; ++j) {
        double nn = 0.0;
        for (int i = lane; i < m; i += kRkWp) nn = fma(a[j * m + i], a[j * m + i], nn);
        nn = dpp::wave_sum(nn);
        if (lane == 0) s[j] = sqrt(nn);
    }
    __syncthreads();
    // selection sort by decreasing s (n <= 4), moving columns and V columns
    for (int j = 0; j < n - 1; ++j) {
        int best = j;
        for (int k = j + 1; k < n; ++k)
            if (s[k] > s[best]) best = k;
        if (best != j) {
            for (int i = lane; i < m; i += kRkWp) {
                const double x = a[j * m + i];
                a[j * m + i] = a[best * m + i];
                a[best * m + i] = x;
            }
            if (lane < n) {
                const double x = V[lane * n + j];
                V[lane * n + j] = V[lane * n + best];
                V[lane * n + best] = x;
            }
            __syncthreads();
            if (lane == 0) {
                const double x = s[j];
                s[j] = s[best];
                s[best] = x;
            }
        }
        __syncthreads();
    }
}

// Weight passing on one network per block.  T (in/out): the network's site
// tensors, chi^rank each at kRkSite strides; S (out): weights per bond,
// decreasing; out_log: the carried log-scale; out_sweeps, status.
template <int CHI>
__global__ void __launch_bounds__(kRkWp) k_weight_pass(const RkGeo *__restrict__ geo_p, double *__restrict__ T_all,
                                                       double *__restrict__ S_all, double *__restrict__ log_all,
                                                       int *__restrict__ sweeps_all, int *__restrict__ status_all,
                                                       double alpha, int ramp, int max_sweeps, double tol) {
    const RkGeo &geo = *geo_p;
    const int net = blockIdx.x, lane = threadIdx.x;
    constexpr int chi = CHI;  // index arithmetic by a constant
    // site tensors packed at their own sizes (dynamic LDS of toff[n_sites]
    // doubles), so several networks share a CU
    extern __shared__ double Tpack[];
    auto T = [&](int s) { return Tpack + geo.toff[s]; };
    __shared__ double S[kRkBonds][kRkChi];
    __shared__ double a[kRkSite], bm[kRkSite];   // A' and B'^T, column-major (others x chi)
    __shared__ double VA[16], VB[16], VC[16], sA[4], sB[4], sC[4], M[16], WA[16], WB[16], nt[kRkSite];
    __shared__ double pa[4], ph[4];  // S_C^a and S_C^((1-a)/2) of the bond being updated
    __shared__ double change;
    double *Tg = T_all + (size_t)net * kRkSites * kRkSite;
    for (int s = 0; s < geo.n_sites; ++s)
        for (int e = lane; e < tsize(geo.rank[s], chi); e += kRkWp) T(s)[e] = Tg[(size_t)s * kRkSite + e];
    for (int e = lane; e < geo.n_bonds * chi; e += kRkWp) S[e / chi][e % chi] = 1.0;
    double log_scale = 0.0;
    int status = 0, sweep = 0;
    __syncthreads();
    for (sweep = 1; sweep <= max_sweeps; ++sweep) {
        const double al = ramp > 0 ? alpha * fmin(1.0, (double)sweep / ramp) : alpha;
        if (lane == 0) change = 0.0;
        __syncthreads();
        for (int b = 0; b < geo.n_bonds; ++b) {
            const int u = geo.bu[b], lu = geo.bul[b], v = geo.bv[b], lv = geo.bvl[b];
            const int ru = geo.rank[u], rv = geo.rank[v];
            const int mu = tsize(ru - 1, chi), mv = tsize(rv - 1, chi);
            // A'[others, i] with the other legs' weights; column i at a[i * mu]
            for (int e = lane; e < tsize(ru, chi); e += kRkWp) {
                int rem = e, oth = 0, ii = 0;
                double w = 1.0;
                for (int l = ru - 1, mul = 1; l >= 0; --l) {
                    const int dg = rem % chi;
                    rem /= chi;
                    if (l == lu) {
                        ii = dg;
                    } else {
                        oth += dg * mul;
                        mul *= chi;
                        const int ob = geo.leg_bond[u][l];
                        if (ob >= 0) w *= S[ob][dg];
                    }
                }
                a[ii * mu + oth] = T(u)[e] * w;
            }
            for (int e = lane; e < tsize(rv, chi); e += kRkWp) {
                int rem = e, oth = 0, ii = 0;
                double w = 1.0;
                for (int l = rv - 1, mul = 1; l >= 0; --l) {
                    const int dg = rem % chi;
                    rem /= chi;
                    if (l == lv) {
                        ii = dg;
                    } else {
                        oth += dg * mul;
                        mul *= chi;
                        const int ob = geo.leg_bond[v][l];
                        if (ob >= 0) w *= S[ob][dg];
                    }
                }
                bm[ii * mv + oth] = T(v)[e] * w;
            }
            __syncthreads();
            // A' = U_A S_A V_A^T ; B'^T = V_B S_B U_B^T, so U_B = (rotations of B'^T)
            jacobi_svd(a, mu, chi, VA, sA);
            jacobi_svd(bm, mv, chi, VB, sB);
            // M = S_A V_A^T diag(S_b) U_B S_B, column-major in M
            if (lane < chi * chi) {
                const int i = lane % chi, j = lane / chi;
                double x = 0.0;
                for (int k = 0; k < chi; ++k) x = fma(VA[k * chi + i] * S[b][k], VB[k * chi + j], x);
                M[j * chi + i] = sA[i] * x * sB[j];
            }
            __syncthreads();
            jacobi_svd(M, chi, chi, VC, sC);  // M columns now U_C S_C
            const double sgm = sA[chi - 1] > 0.0 && sB[chi - 1] > 0.0 && sC[chi - 1] > 0.0 ? 1.0 : 0.0;
            if (sgm == 0.0) status = PNE_ERR_SINGULAR;
            if (lane < chi) {
                pa[lane] = pow(sC[lane], al);
                ph[lane] = pow(sC[lane], 0.5 * (1.0 - al));
            }
            __syncthreads();
            // W_A = V_A S_A^-1 U_C S_C^((1-a)/2);  W_B = S_C^((1-a)/2) V_C^T S_B^-1 U_B^T
            if (lane < chi * chi) {
                const int i = lane / chi, j = lane % chi;
                const double h = ph[j];
                double x = 0.0;
                for (int k = 0; k < chi; ++k) x = fma(VA[i * chi + k] / sA[k], M[j * chi + k] / sC[j], x);
                WA[i * chi + j] = x * h;
                const double h2 = ph[i];
                double y = 0.0;
                for (int k = 0; k < chi; ++k) y = fma(VC[k * chi + i] / sB[k], VB[j * chi + k], y);
                WB[i * chi + j] = h2 * y;
            }
            __syncthreads();
            // A <- A x_lu W_A ; B <- W_B x_lv B
            for (int e = lane; e < tsize(ru, chi); e += kRkWp) {
                int stride = 1;
                for (int l = ru - 1; l > lu; --l) stride *= chi;
                const int j = (e / stride) % chi, base = e - j * stride;
                double x = 0.0;
                for (int i = 0; i < chi; ++i) x = fma(T(u)[base + i * stride], WA[i * chi + j], x);
                nt[e] = x;
            }
            __syncthreads();
            for (int e = lane; e < tsize(ru, chi); e += kRkWp) T(u)[e] = nt[e];
            __syncthreads();
            for (int e = lane; e < tsize(rv, chi); e += kRkWp) {
                int stride = 1;
                for (int l = rv - 1; l > lv; --l) stride *= chi;
                const int j = (e / stride) % chi, base = e - j * stride;
                double x = 0.0;
                for (int i = 0; i < chi; ++i) x = fma(WB[j * chi + i], T(v)[base + i * stride], x);
                nt[e] = x;
            }
            __syncthreads();
            for (int e = lane; e < tsize(rv, chi); e += kRkWp) T(v)[e] = nt[e];
            double mx = 0.0;
            for (int k = 0; k < chi; ++k) mx = fmax(mx, pa[k]);
            if (lane == 0) {
                double ch = change;
                for (int k = 0; k < chi; ++k) {
                    const double nw = pa[k] / mx;
                    ch = fmax(ch, fabs(nw - S[b][k]));
                    S[b][k] = nw;
                }
                change = ch;
            }
            log_scale += log(mx);
            __syncthreads();
        }
        const bool done = change <= tol && sweep >= ramp;
        __syncthreads();
        if (done || status) break;
    }
    if (sweep > max_sweeps) {
        sweep = max_sweeps;
        if (!status) status = PNE_WARN_BP_NOT_CONVERGED;
    }
    for (int s = 0; s < geo.n_sites; ++s)
        for (int e = lane; e < tsize(geo.rank[s], chi); e += kRkWp) Tg[(size_t)s * kRkSite + e] = T(s)[e];
    for (int e = lane; e < geo.n_bonds * chi; e += kRkWp)
        S_all[(size_t)net * kRkBonds * kRkChi + (e / chi) * kRkChi + e % chi] = S[e / chi][e % chi];
    if (lane == 0) {
        log_all[net] = log_scale;
        sweeps_all[net] = sweep;
        status_all[net] = status;
    }
}

// One term of one network per block: the gauged lattice contracted site by
// site in row-major order with a diagonal operator on every bond
// (op code per bond: 0 whole weight, 1 its first r entries (P), 2 the rest
// (Q)), applied when the bond's first (left or upper) site is absorbed.  The
// state holds the horizontal leg h and one vertical index per column, chi each
// (index 0 only where a leg does not exist); each row ends with a rescale
// whose log is carried.  out[term] = (log, value).
__global__ void __launch_bounds__(256) k_lattice_terms(const RkGeo *__restrict__ geo_p,
                                                       const double *__restrict__ T_all,
                                                       const double *__restrict__ S_all,
                                                       const int8_t *__restrict__ ops, int n_terms, int r,
                                                       double *__restrict__ out) {
    const RkGeo &geo = *geo_p;
    const int net = blockIdx.x / n_terms, term = blockIdx.x % n_terms, tid = threadIdx.x;
    const int chi = geo.chi, Lx = geo.Lx;
    __shared__ double st[2][kRkState];
    __shared__ double site[kRkSite];
    __shared__ double dR[kRkChi], dD[kRkChi];
    __shared__ double red[4];
    const double *Tn = T_all + (size_t)net * kRkSites * kRkSite;
    const double *Sn = S_all + (size_t)net * kRkBonds * kRkChi;
    const int8_t *op = ops + (size_t)term * geo.n_bonds;
    int ncol = 1;
    for (int x = 0; x < Lx; ++x) ncol *= chi;
    const int nst = chi * ncol;  // [h][c_0 .. c_{Lx-1}]
    for (int e = tid; e < nst; e += 256) st[0][e] = e == 0 ? 1.0 : 0.0;
    int cur = 0;
    double log_acc = 0.0;
    __syncthreads();
    for (int y = 0; y < geo.Ly; ++y) {
        for (int x = 0; x < Lx; ++x) {
            const int s = x + Lx * y;
            for (int e = tid; e < tsize(geo.rank[s], chi); e += 256) site[e] = Tn[(size_t)s * kRkSite + e];
            if (tid < chi) {
                for (int k = 0; k < 2; ++k) {
                    const int sl = geo.dir_slot[s][k == 0 ? 1 : 3];
                    double d = 1.0;
                    if (sl >= 0) {
                        const int b = geo.leg_bond[s][sl];
                        const int code = op[b];
                        d = Sn[b * kRkChi + tid];
                        if ((code == 1 && tid >= r) || (code == 2 && tid < r)) d = 0.0;
                    } else if (tid > 0) {
                        d = 0.0;
                    }
                    (k == 0 ? dR : dD)[tid] = d;
                }
            }
            __syncthreads();
            const int sl_l = geo.dir_slot[s][0], sl_r = geo.dir_slot[s][1], sl_u = geo.dir_slot[s][2],
                      sl_d = geo.dir_slot[s][3];
            int colstride = 1;
            for (int k = Lx - 1; k > x; --k) colstride *= chi;
            const int rank = geo.rank[s];
            for (int e = tid; e < nst; e += 256) {
                const int h2 = e / ncol, rest = e % ncol;
                const int c2 = (rest / colstride) % chi;
                const int base = rest - c2 * colstride;
                double acc = 0.0;
                if (dR[h2] != 0.0 && dD[c2] != 0.0) {
                    const int hmax = sl_l >= 0 ? chi : 1, cmax = sl_u >= 0 ? chi : 1;
                    for (int h = 0; h < hmax; ++h)
                        for (int c = 0; c < cmax; ++c) {
                            int idx = 0;
                            for (int l = 0; l < rank; ++l) {
                                const int dg = l == sl_l ? h : l == sl_r ? h2 : l == sl_u ? c : c2;
                                idx = idx * chi + dg;
                            }
                            acc = fma(st[cur][h * ncol + base + c * colstride], site[idx], acc);
                        }
                    acc *= dR[h2] * dD[c2];
                }
                st[cur ^ 1][e] = acc;
            }
            cur ^= 1;
            __syncthreads();
        }
        // rescale by the largest magnitude
        double mx = 0.0;
        for (int e = tid; e < nst; e += 256) mx = fmax(mx, fabs(st[cur][e]));
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        if ((tid & 63) == 0) red[tid >> 6] = mx;
        __syncthreads();
        mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        if (mx > 0.0) {
            for (int e = tid; e < nst; e += 256) st[cur][e] /= mx;
            log_acc += log(mx);
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[2 * (size_t)blockIdx.x] = log_acc;
        out[2 * (size_t)blockIdx.x + 1] = st[cur][0];
    }
}

}  // namespace

// Per network: sum_t sign_t v_t exp(log_t - ref) in FP64, plus the
// weight-passing log-scale.
__global__ void k_rank_combine(const double *__restrict__ terms, const int8_t *__restrict__ sgn, int n_terms,
                               int n_nets, const double *__restrict__ log_all, pne_rank_result *__restrict__ res,
                               const int *__restrict__ sweeps_all, const int *__restrict__ status_all) {
    const int net = blockIdx.x * blockDim.x + threadIdx.x;
    if (net >= n_nets) return;
    const double *t = terms + 2 * (size_t)net * n_terms;
    double ref = -INFINITY;
    for (int k = 0; k < n_terms; ++k)
        if (t[2 * k + 1] != 0.0) ref = fmax(ref, t[2 * k] + log(fabs(t[2 * k + 1])));
    double tot = 0.0;
    if (ref > -INFINITY)
        for (int k = 0; k < n_terms; ++k)
            if (t[2 * k + 1] != 0.0) tot += sgn[k] * t[2 * k + 1] * exp(t[2 * k] - ref);
    pne_rank_result r;
    r.status = status_all[net];
    r.sweeps = sweeps_all[net];
    r.sign = tot > 0.0 ? 1 : (tot < 0.0 ? -1 : 0);
    r.pad = 0;
    r.log_abs = tot == 0.0 ? -INFINITY : ref + log(fabs(tot)) + log_all[net];
    r.log_scale = log_all[net];
    res[net] = r;
}

namespace {

// Gather the networks' site tensors into the padded layout [net][site][kRkSite].
__global__ void k_rank_gather(const double *const *__restrict__ src, const int *__restrict__ sizes, int n_sites,
                              double *__restrict__ T_all) {
    const int net = blockIdx.x;
    for (int s = 0; s < n_sites; ++s) {
        const double *p = src[(size_t)net * n_sites + s];
        for (int e = threadIdx.x; e < sizes[s]; e += blockDim.x)
            T_all[((size_t)net * kRkSites + s) * kRkSite + e] = gld(p + e);
    }
}

}  // namespace
}  // namespace pne

using namespace pne;

extern "C" pne_status pne_rank_options_default(pne_rank_options *opt) {
    if (!opt) return PNE_ERR_INVALID_ARG;
    std::memset(opt, 0, sizeof *opt);
    opt->rank = 2;
    opt->form = 0;
    opt->alpha = 0.8;
    opt->ramp_sweeps = 10;
    opt->max_sweeps = 2000;
    opt->tol = 1e-12;
    return PNE_OK;
}

extern "C" pne_status pne_rank_last_times(pne_ctx *ctx, double *ms, int32_t n) {
    if (!ctx || !ms || n < 0 || n > 5) return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "need ctx, ms and 0 <= n <= 5");
    for (int k = 0; k < n; ++k) ms[k] = ctx_rank_times(ctx)[k];
    return PNE_OK;
}

extern "C" pne_status pne_rank_expand(pne_ctx *ctx, pne_network *const *nets, int32_t n, int32_t Lx, int32_t Ly,
                                      int32_t n_partitions, const int32_t *part_begin, const int32_t *part_bond,
                                      const pne_rank_options *opt, pne_rank_result *results) {
    if (!ctx || !nets || n < 1 || !opt || !results || !part_begin || (n_partitions > 0 && !part_bond))
        return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "null or empty argument");
    for (int k = 0; k < 5; ++k) ctx_rank_times(ctx)[k] = 0.0;
    if (Lx < 1 || Ly < 1 || Lx * Ly > kRkSites)
        return ctx_fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: lattice of more than 16 sites");
    if (n_partitions < 1 || n_partitions > 16)
        return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "need 1..16 partitions");
    if (opt->form != 0 && opt->form != 1) return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "form must be 0 or 1");
    if (!(opt->alpha > 0.0 && opt->alpha <= 1.0) || opt->max_sweeps < 1 || opt->ramp_sweeps < 0)
        return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "alpha in (0, 1], max_sweeps >= 1, ramp_sweeps >= 0");
    // geometry: every network a closed Lx x Ly lattice, sites x + Lx y, one bond dimension
    RkGeo geo;
    std::memset(&geo, 0, sizeof geo);
    const int n_sites = network_sites(nets[0]);
    if (n_sites != Lx * Ly) return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "site count is not Lx * Ly");
    std::vector<int> rank, bu, bul, bv, bvl, dims;
    if (!network_graph(nets[0], &rank, &dims, &bu, &bul, &bv, &bvl))
        return ctx_fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: networks with open legs");
    const int chi = dims.empty() ? 0 : dims[0];
    for (int d : dims)
        if (d != chi) return ctx_fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: bond dimensions differ");
    // chi <= 4: the one-wave kernels below; chi 8 or 16: the MFMA path (rankr_large.hip)
    const bool large = chi > kRkChi;
    if (chi < 1 || (large && !rank_large_supported(chi, Lx, Ly)))
        return ctx_fail(ctx, PNE_ERR_UNSUPPORTED,
                        "unsupported: bond dimension above 4 needs chi in {8, 16}, Lx >= 2, chi^(Lx-1) a multiple "
                        "of 16 and chi^(Lx+1) <= 65536");
    int ncol = 1;
    for (int x = 0; x <= Lx; ++x) ncol *= chi;
    if (!large && ncol > kRkState) return ctx_fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: chi^(Lx+1) above 1024");
    for (int i = 1; i < n; ++i)
        if (!same_geometry(nets[0], nets[i])) return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "networks differ in geometry");
    const int nb = (int)bu.size();
    if (nb > kRkBonds) return ctx_fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: too many bonds");
    geo.n_sites = n_sites;
    geo.n_bonds = nb;
    geo.chi = chi;
    geo.Lx = Lx;
    geo.Ly = Ly;
    geo.toff[0] = 0;
    for (int s = 0; s < n_sites; ++s) {
        geo.rank[s] = rank[s];
        for (int l = 0; l < 4; ++l) geo.leg_bond[s][l] = geo.dir_slot[s][l] = -1;
        int z = 1;
        for (int l = 0; l < rank[s]; ++l) z *= chi;
        geo.toff[s + 1] = geo.toff[s] + z;
    }
    for (int b = 0; b < nb; ++b) {
        int u = bu[b], lu = bul[b], v = bv[b], lv = bvl[b];
        if (v < u) {
            std::swap(u, v);
            std::swap(lu, lv);
        }
        const int ux = u % Lx, uy = u / Lx, vx = v % Lx, vy = v / Lx;
        int du, dv;
        if (vy == uy && vx == ux + 1) {
            du = 1;
            dv = 0;
        } else if (vx == ux && vy == uy + 1) {
            du = 3;
            dv = 2;
        } else {
            return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "a bond does not join lattice neighbours");
        }
        if (geo.dir_slot[u][du] >= 0 || geo.dir_slot[v][dv] >= 0)
            return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "two bonds in one direction");
        geo.dir_slot[u][du] = lu;
        geo.dir_slot[v][dv] = lv;
        geo.leg_bond[u][lu] = b;
        geo.leg_bond[v][lv] = b;
        geo.bu[b] = bu[b];
        geo.bul[b] = bul[b];
        geo.bv[b] = bv[b];
        geo.bvl[b] = bvl[b];
    }
    if (opt->rank < 1 || opt->rank > chi) return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "rank must be in [1, chi]");
    // terms: op code per bond (0 whole weight, 1 P, 2 Q) and sign
    std::vector<std::vector<int>> parts(n_partitions);
    if (part_begin[0] != 0) return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "partition offsets must start at 0");
    for (int p = 0; p < n_partitions; ++p) {
        if (part_begin[p + 1] <= part_begin[p]) return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "empty partition");
        for (int k = part_begin[p]; k < part_begin[p + 1]; ++k) {
            if (part_bond[k] < 0 || part_bond[k] >= nb) return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "bond out of range");
            parts[p].push_back(part_bond[k]);
        }
    }
    std::vector<int8_t> ops, sgn;
    int n_terms = 0;
    if (opt->form == 0) {
        for (uint32_t x = 1; x < (1u << n_partitions); ++x) {
            std::vector<int8_t> o(nb, 0);
            for (int p = 0; p < n_partitions; ++p)
                if (x >> p & 1)
                    for (int b : parts[p]) o[b] = 1;
            ops.insert(ops.end(), o.begin(), o.end());
            sgn.push_back((__builtin_popcount(x) & 1) ? 1 : -1);
            ++n_terms;
        }
    } else {
        for (int p = 0; p < n_partitions; ++p)
            if (parts[p].size() != 1)
                return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "the linear form takes single-index partitions");
        for (int k = 0; k < n_partitions; ++k) {
            std::vector<int8_t> o(nb, 0);
            for (int q = 0; q < k; ++q) o[parts[q][0]] = 2;
            o[parts[k][0]] = 1;
            ops.insert(ops.end(), o.begin(), o.end());
            sgn.push_back(1);
            ++n_terms;
        }
    }
    RankTimer timer(opt->profile != 0);
    if (large) return rank_expand_large(ctx, nets, n, geo, ops, sgn, n_terms, opt, results, timer);
    hipStream_t s = ctx_stream(ctx);
    // device buffers in one allocation
    std::vector<const double *> src((size_t)n * n_sites);
    for (int i = 0; i < n; ++i)
        for (int q = 0; q < n_sites; ++q) src[(size_t)i * n_sites + q] = network_site_ptr(nets[i], q);
    std::vector<int> sizes(n_sites);
    for (int q = 0; q < n_sites; ++q) {
        int z = 1;
        for (int l = 0; l < rank[q]; ++l) z *= chi;
        sizes[q] = z;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t oGeo = take(sizeof(RkGeo)), oSrc = take(src.size() * sizeof(double *)),
                 oSizes = take(sizes.size() * sizeof(int)), oT = take((size_t)n * kRkSites * kRkSite * 8),
                 oS = take((size_t)n * kRkBonds * kRkChi * 8), oLog = take((size_t)n * 8), oSw = take((size_t)n * 4),
                 oSt = take((size_t)n * 4), oOps = take(ops.size()), oSgn = take(sgn.size()),
                 oTerms = take((size_t)n * n_terms * 2 * 8), oRes = take((size_t)n * sizeof(pne_rank_result));
    void *buf = nullptr;
    if (hipMalloc(&buf, off) != hipSuccess) return ctx_fail(ctx, PNE_ERR_OUT_OF_MEMORY, "rank expansion: hipMalloc failed");
    char *B = static_cast<char *>(buf);
    pne_status st = PNE_OK;
    auto fin = [&](pne_status r) {
        (void)hipFree(buf);
        return r;
    };
#define RK_TRY(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fin(ctx_fail(ctx, PNE_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_))); \
    } while (0)
    RK_TRY(hipMemcpyAsync(B + oGeo, &geo, sizeof geo, hipMemcpyHostToDevice, s));
    RK_TRY(hipMemcpyAsync(B + oSrc, src.data(), src.size() * sizeof(double *), hipMemcpyHostToDevice, s));
    RK_TRY(hipMemcpyAsync(B + oSizes, sizes.data(), sizes.size() * sizeof(int), hipMemcpyHostToDevice, s));
    RK_TRY(hipMemcpyAsync(B + oOps, ops.data(), ops.size(), hipMemcpyHostToDevice, s));
    RK_TRY(hipMemcpyAsync(B + oSgn, sgn.data(), sgn.size(), hipMemcpyHostToDevice, s));
    timer.mark(s);
    hipLaunchKernelGGL(k_rank_gather, dim3(n), dim3(256), 0, s, reinterpret_cast<const double *const *>(B + oSrc),
                       reinterpret_cast<const int *>(B + oSizes), n_sites, reinterpret_cast<double *>(B + oT));
    RK_TRY(hipGetLastError());
    timer.mark(s);
    {
        const size_t lds = (size_t)geo.toff[n_sites] * sizeof(double);
        auto *g = reinterpret_cast<const RkGeo *>(B + oGeo);
        auto *T = reinterpret_cast<double *>(B + oT);
        auto *Sw = reinterpret_cast<double *>(B + oS);
        auto *Lg = reinterpret_cast<double *>(B + oLog);
        auto *Sp = reinterpret_cast<int *>(B + oSw);
        auto *St = reinterpret_cast<int *>(B + oSt);
        switch (chi) {
            case 1:
                hipLaunchKernelGGL(k_weight_pass<1>, dim3(n), dim3(kRkWp), lds, s, g, T, Sw, Lg, Sp, St, opt->alpha,
                                   opt->ramp_sweeps, opt->max_sweeps, opt->tol);
                break;
            case 2:
                hipLaunchKernelGGL(k_weight_pass<2>, dim3(n), dim3(kRkWp), lds, s, g, T, Sw, Lg, Sp, St, opt->alpha,
                                   opt->ramp_sweeps, opt->max_sweeps, opt->tol);
                break;
            case 3:
                hipLaunchKernelGGL(k_weight_pass<3>, dim3(n), dim3(kRkWp), lds, s, g, T, Sw, Lg, Sp, St, opt->alpha,
                                   opt->ramp_sweeps, opt->max_sweeps, opt->tol);
                break;
            default:
                hipLaunchKernelGGL(k_weight_pass<4>, dim3(n), dim3(kRkWp), lds, s, g, T, Sw, Lg, Sp, St, opt->alpha,
                                   opt->ramp_sweeps, opt->max_sweeps, opt->tol);
                break;
        }
    }
    RK_TRY(hipGetLastError());
    timer.mark(s);
    timer.mark(s);  // no site-matrix phase at chi <= 4
    hipLaunchKernelGGL(k_lattice_terms, dim3((unsigned)n * n_terms), dim3(256), 0, s,
                       reinterpret_cast<const RkGeo *>(B + oGeo), reinterpret_cast<const double *>(B + oT),
                       reinterpret_cast<const double *>(B + oS), reinterpret_cast<const int8_t *>(B + oOps), n_terms,
                       opt->rank, reinterpret_cast<double *>(B + oTerms));
    RK_TRY(hipGetLastError());
    timer.mark(s);
    hipLaunchKernelGGL(k_rank_combine, dim3((n + 63) / 64), dim3(64), 0, s, reinterpret_cast<const double *>(B + oTerms),
                       reinterpret_cast<const int8_t *>(B + oSgn), n_terms, n, reinterpret_cast<const double *>(B + oLog),
                       reinterpret_cast<pne_rank_result *>(B + oRes), reinterpret_cast<const int *>(B + oSw),
                       reinterpret_cast<const int *>(B + oSt));
    RK_TRY(hipGetLastError());
    timer.mark(s);
    RK_TRY(hipMemcpyAsync(results, B + oRes, (size_t)n * sizeof(pne_rank_result), hipMemcpyDeviceToHost, s));
    RK_TRY(hipStreamSynchronize(s));
#undef RK_TRY
    timer.read(ctx_rank_times(ctx), 5);
    for (int i = 0; i < n; ++i) {
        if (results[i].status < 0 && st == PNE_OK) st = (pne_status)results[i].status;
        else if (results[i].status > 0 && st == PNE_OK) st = (pne_status)results[i].status;
    }
    return fin(st);
}
