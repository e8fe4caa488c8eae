// Rank-r projectors from weight passing (Sec. V, Appendix C) at the paper's
// bond dimensions (chi = 8 or 16; Sec. V.B coarse-grains 12 x 12 Ising
// lattices into 3 x 3 sites of chi = 16).
//
//   k_wpl           weight passing, one 256-thread block per network, site
//                   tensors in global memory (a chi = 16 centre site is 512 KB).
//                   Each bond update (Eqs. (C1)-(C3)) needs only the singular
//                   values and right vectors of the weighted site matrices:
//                   a Householder QR of the (others x chi) matrix reduces it to
//                   its chi x chi R factor, whose SVD (parallel one-sided
//                   Jacobi, round-robin pairs) gives S and V; the chi x chi core
//                   of Eq. (C2) is decomposed the same way.
//   k_pad_sites     each site as a dense (h, c) x (h', c') matrix (legs -x, -y
//                   by legs +x, +y; an absent leg keeps only index 0).
//   k_terms_mfma    every term of the expansion: the lattice contracted row by
//                   row, one site at a time.  Absorbing a site is a dense GEMM
//                   (other columns) x (h, c) by (h, c) x (h', c'), 256^3 at
//                   chi = 16 on a 3-wide lattice, run on the FP64 matrix cores
//                   (v_mfma_f64_16x16x4f64) with the bond operators of the term
//                   applied to the output columns.  Structurally zero k-steps
//                   (absent legs) are skipped.
//   k_rank_combine  the signed FP64 sum of the terms (shared with rankr.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gmem.h"
#include "pne.h"
#include "rankr.h"
#include "runtime.h"

namespace pne {
namespace {

using dev::gld;

constexpr int kLt = 256;  // threads of the weight-passing and term blocks (four waves)
typedef double double4_t __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int ipow_l(int b, int e) { return e <= 0 ? 1 : b * ipow_l(b, e - 1); }

// Sum of NV values per thread over the block, fixed order (red: 4 * NV doubles).
template <int NV>
__device__ inline void block_sum_vec(double (&v)[NV], double *red) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
        v[k] = x;
    }
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = (red[k] + red[NV + k]) + (red[2 * NV + k] + red[3 * NV + k]);
    __syncthreads();
}

__device__ inline double block_max(double v, double *red) {
    const int tid = threadIdx.x;
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    v = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return v;
}

// Householder QR of the m x CHI column-major matrix a (global, column j at
// a + j * m, m >= CHI), by the block.  R (row-major, CHI x CHI, upper
// triangle) goes to LDS; a is overwritten by the reflectors.
template <int CHI>
__device__ void house_qr(double *a, int m, double *R, double *red) {
    const int tid = threadIdx.x;
    for (int j = 0; j < CHI; ++j) {
        double *aj = a + (size_t)j * m;
        double nv[1] = {0.0};
        for (int i = j + tid; i < m; i += kLt) nv[0] = fma(aj[i], aj[i], nv[0]);
        block_sum_vec<1>(nv, red);
        const double nrm2 = nv[0];
        const double x0 = aj[j];
        const double nrm = sqrt(nrm2);
        const double alpha = nrm == 0.0 ? 0.0 : (x0 >= 0.0 ? -nrm : nrm);
        const double v0 = x0 - alpha;
        const double vn2 = nrm2 - x0 * x0 + v0 * v0;
        const double tau = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
        __syncthreads();  // every thread has read x0
        if (tid == 0) aj[j] = v0;
        __syncthreads();
        double d[CHI];
#pragma unroll
        for (int k = 0; k < CHI; ++k) d[k] = 0.0;
        for (int i = j + tid; i < m; i += kLt) {
            const double vi = aj[i];
#pragma unroll
            for (int k = 0; k < CHI; ++k)
                if (k > j) d[k] = fma(vi, a[(size_t)k * m + i], d[k]);
        }
        block_sum_vec<CHI>(d, red);
        for (int i = j + tid; i < m; i += kLt) {
            const double vi = aj[i];
#pragma unroll
            for (int k = 0; k < CHI; ++k)
                if (k > j) a[(size_t)k * m + i] -= tau * d[k] * vi;
        }
        __syncthreads();
        if (tid < CHI) R[j * CHI + tid] = tid < j ? 0.0 : (tid == j ? alpha : a[(size_t)tid * m + j]);
        __syncthreads();
    }
}

// One-sided Jacobi SVD of the CHI x CHI matrix W (LDS, column-major: column q
// at W + q * CHI), by the block: disjoint column pairs of a round-robin
// schedule rotate in parallel, 16 lanes per pair.  On return the columns of W
// are U S, V (row-major, V[i * CHI + j]) holds the rotations, s the column
// norms, all sorted by decreasing s.  Rotations stop once every pair is
// orthogonal to 1e-15 relative, or after 60 sweeps.  perm, flag: LDS scratch;
// tmp: LDS scratch of 2 * CHI * CHI doubles.
template <int CHI>
__device__ void jacobi_small(double *W, double *V, double *s, int *perm, int *flag, double *tmp) {
    constexpr int NP = (CHI + 1) & ~1;  // players of the round-robin schedule (one dummy if CHI is odd)
    const int tid = threadIdx.x, g = tid >> 4, l = tid & 15;
    for (int e = tid; e < CHI * CHI; e += kLt) V[e] = (e / CHI == e % CHI) ? 1.0 : 0.0;
    __syncthreads();
    for (int sweep = 0; sweep < 60; ++sweep) {
        if (tid == 0) *flag = 0;
        __syncthreads();
        for (int r = 0; r < NP - 1; ++r) {
            if (g < NP / 2) {
                auto pos = [&](int i) { return i == 0 ? 0 : 1 + (i - 1 + r) % (NP - 1); };
                int p = pos(g), q = pos(NP - 1 - g);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                const bool real = q < CHI;
                const double x = (real && l < CHI) ? W[p * CHI + l] : 0.0;
                const double y = (real && l < CHI) ? W[q * CHI + l] : 0.0;
                double al = x * x, be = y * y, ga = x * y;
                for (int o = 8; o > 0; o >>= 1) {
                    al += __shfl_xor(al, o, 16);
                    be += __shfl_xor(be, o, 16);
                    ga += __shfl_xor(ga, o, 16);
                }
                // The butterfly's sums can differ in the last bit from lane to
                // lane (the first step may fuse into an FMA), and with tied
                // column norms that flips the sign of be - al, and so of the
                // rotation, between lanes: every lane takes the first lane's.
                al = __shfl(al, 0, 16);
                be = __shfl(be, 0, 16);
                ga = __shfl(ga, 0, 16);
                if (real && ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                    if (l < CHI) {
                        W[p * CHI + l] = c * x - sn * y;
                        W[q * CHI + l] = sn * x + c * y;
                        const double vx = V[l * CHI + p], vy = V[l * CHI + q];
                        V[l * CHI + p] = c * vx - sn * vy;
                        V[l * CHI + q] = sn * vx + c * vy;
                    }
                    if (l == 0) *flag = 1;  // every writer stores the same value
                }
            }
            __syncthreads();
        }
        const int rotated = *flag;
        __syncthreads();
        if (!rotated) break;
    }
    if (tid < CHI) {
        double nn = 0.0;
        for (int i = 0; i < CHI; ++i) nn = fma(W[tid * CHI + i], W[tid * CHI + i], nn);
        s[tid] = sqrt(nn);
    }
    __syncthreads();
    if (tid == 0) {  // order by decreasing s (ties keep the column order)
        for (int j = 0; j < CHI; ++j) perm[j] = j;
        for (int j = 0; j < CHI - 1; ++j) {
            int best = j;
            for (int k = j + 1; k < CHI; ++k)
                if (s[perm[k]] > s[perm[best]]) best = k;
            const int t = perm[j];
            perm[j] = perm[best];
            perm[best] = t;
        }
    }
    __syncthreads();
    for (int e = tid; e < CHI * CHI; e += kLt) {
        const int col = e / CHI, row = e % CHI;
        tmp[e] = W[perm[col] * CHI + row];                            // column col of the sorted W
        tmp[CHI * CHI + row * CHI + col] = V[row * CHI + perm[col]];  // V, columns permuted
    }
    double sv = 0.0;
    if (tid < CHI) sv = s[perm[tid]];
    __syncthreads();
    for (int e = tid; e < CHI * CHI; e += kLt) {
        W[e] = tmp[e];
        V[e] = tmp[CHI * CHI + e];
    }
    if (tid < CHI) s[tid] = sv;
    __syncthreads();
}

// Weight passing on one network per block (Eqs. (C1)-(C3)); same update and
// stopping rule as the small-chi kernel in rankr.hip.  T (in/out): the
// network's site tensors packed at geo.toff; scr: 3 * chi^3 * chi doubles of
// per-network scratch (the two weighted site matrices and a mode-product
// buffer).
template <int CHI>
__global__ void __launch_bounds__(kLt) k_wpl(const RkGeo *__restrict__ geo_p, double *__restrict__ T_all,
                                               int64_t net_stride, double *__restrict__ scr_all,
                                               int64_t scr_stride, double *__restrict__ S_all,
                                               double *__restrict__ log_all, int *__restrict__ sweeps_all,
                                               int *__restrict__ status_all, double alpha, int ramp, int max_sweeps,
                                               double tol) {
    const RkGeo &geo = *geo_p;
    const int net = blockIdx.x, tid = threadIdx.x;
    double *T = T_all + (size_t)net * net_stride;
    double *a = scr_all + (size_t)net * scr_stride;
    const int64_t mmax = (int64_t)ipow_l(CHI, 3) * CHI;
    double *bm = a + mmax;
    double *nt = bm + mmax;
    __shared__ double S[kRkBonds][CHI];
    __shared__ double R[CHI * CHI], W[CHI * CHI], VA[CHI * CHI], VB[CHI * CHI], VC[CHI * CHI];
    __shared__ double WA[CHI * CHI], WB[CHI * CHI], tmp[2 * CHI * CHI];
    __shared__ double sA[CHI], sB[CHI], sC[CHI], pa[CHI], ph[CHI], red[4 * CHI];
    __shared__ int perm[CHI], flag;
    __shared__ double change;
    for (int e = tid; e < geo.n_bonds * CHI; e += kLt) S[e / CHI][e % CHI] = 1.0;
    double log_scale = 0.0;
    int status = 0, sweep = 0;
    __syncthreads();
    auto build = [&](int site, int leg, double *dst) {
        // site matrix (others x chi), column-major, with the other bonds' weights
        const int rk = geo.rank[site];
        const int m = ipow_l(CHI, rk - 1);
        const double *t = T + geo.toff[site];
        for (int e = tid; e < m * CHI; e += kLt) {
            int rem = e, oth = 0, ii = 0, mul = 1;
            double w = 1.0;
            for (int l = rk - 1; l >= 0; --l) {
                const int dg = rem % CHI;
                rem /= CHI;
                if (l == leg) {
                    ii = dg;
                } else {
                    oth += dg * mul;
                    mul *= CHI;
                    const int ob = geo.leg_bond[site][l];
                    if (ob >= 0) w *= S[ob][dg];
                }
            }
            dst[(size_t)ii * m + oth] = t[e] * w;
        }
        __syncthreads();
        return m;
    };
    for (sweep = 1; sweep <= max_sweeps; ++sweep) {
        const double al = ramp > 0 ? alpha * fmin(1.0, (double)sweep / ramp) : alpha;
        if (tid == 0) change = 0.0;
        __syncthreads();
        for (int b = 0; b < geo.n_bonds && !status; ++b) {
            const int u = geo.bu[b], lu = geo.bul[b], v = geo.bv[b], lv = geo.bvl[b];
            // A' = U_A S_A V_A^T: S_A, V_A from the SVD of A' = Q R's factor R
            const int mu = build(u, lu, a);
            house_qr<CHI>(a, mu, R, red);
            for (int e = tid; e < CHI * CHI; e += kLt) W[(e % CHI) * CHI + e / CHI] = R[e];
            __syncthreads();
            jacobi_small<CHI>(W, VA, sA, perm, &flag, tmp);
            // B'^T = V_B S_B U_B^T: S_B, U_B from the SVD of B'^T's R factor
            const int mv = build(v, lv, bm);
            house_qr<CHI>(bm, mv, R, red);
            for (int e = tid; e < CHI * CHI; e += kLt) W[(e % CHI) * CHI + e / CHI] = R[e];
            __syncthreads();
            jacobi_small<CHI>(W, VB, sB, perm, &flag, tmp);
            // core M = S_A V_A^T diag(S_b) U_B S_B (column-major in W), then its SVD
            for (int e = tid; e < CHI * CHI; e += kLt) {
                const int i = e % CHI, j = e / CHI;
                double x = 0.0;
                for (int k = 0; k < CHI; ++k) x = fma(VA[k * CHI + i] * S[b][k], VB[k * CHI + j], x);
                W[j * CHI + i] = sA[i] * x * sB[j];
            }
            __syncthreads();
            jacobi_small<CHI>(W, VC, sC, perm, &flag, tmp);  // W columns: U_C S_C
            if (!(sA[CHI - 1] > 0.0 && sB[CHI - 1] > 0.0 && sC[CHI - 1] > 0.0)) {
                status = PNE_ERR_SINGULAR;
                break;
            }
            if (tid < CHI) {
                pa[tid] = pow(sC[tid], al);
                ph[tid] = pow(sC[tid], 0.5 * (1.0 - al));
            }
            __syncthreads();
            // W_A = V_A S_A^-1 U_C S_C^((1-a)/2);  W_B = S_C^((1-a)/2) V_C^T S_B^-1 U_B^T
            for (int e = tid; e < CHI * CHI; e += kLt) {
                const int i = e / CHI, j = e % CHI;
                double x = 0.0;
                for (int k = 0; k < CHI; ++k) x = fma(VA[i * CHI + k] / sA[k], W[j * CHI + k] / sC[j], x);
                WA[i * CHI + j] = x * ph[j];
                double y = 0.0;
                for (int k = 0; k < CHI; ++k) y = fma(VC[k * CHI + i] / sB[k], VB[j * CHI + k], y);
                WB[i * CHI + j] = ph[i] * y;
            }
            __syncthreads();
            // A <- A x_lu W_A ; B <- W_B x_lv B (through the mode-product buffer)
            for (int side = 0; side < 2; ++side) {
                const int site = side ? v : u, leg = side ? lv : lu, rk = geo.rank[site];
                double *t = T + geo.toff[site];
                int stride = 1;
                for (int l = rk - 1; l > leg; --l) stride *= CHI;
                const int size = ipow_l(CHI, rk);
                for (int e = tid; e < size; e += kLt) {
                    const int j = (e / stride) % CHI, base = e - j * stride;
                    double x = 0.0;
                    for (int i = 0; i < CHI; ++i)
                        x = fma(t[base + i * stride], side ? WB[j * CHI + i] : WA[i * CHI + j], x);
                    nt[e] = x;
                }
                __syncthreads();
                for (int e = tid; e < size; e += kLt) t[e] = nt[e];
                __syncthreads();
            }
            double mx = 0.0;
            for (int k = 0; k < CHI; ++k) mx = fmax(mx, pa[k]);
            if (tid == 0) {
                double ch = change;
                for (int k = 0; k < CHI; ++k) {
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
    for (int e = tid; e < geo.n_bonds * CHI; e += kLt)
        S_all[(size_t)net * kRkBonds * kRkLargeChi + (e / CHI) * kRkLargeChi + e % CHI] = S[e / CHI][e % CHI];
    if (tid == 0) {
        log_all[net] = log_scale;
        sweeps_all[net] = sweep;
        status_all[net] = status;
    }
}

// Site s of network net as the dense matrix P[k][n], k = h * chi + c over
// (-x, -y) and n = h' * chi + c' over (+x, +y); an absent leg contributes
// index 0 only.  One block per (network, site).
template <int CHI>
__global__ void __launch_bounds__(kLt) k_pad_sites(const RkGeo *__restrict__ geo_p, const double *__restrict__ T_all,
                                                     int64_t net_stride, double *__restrict__ P_all) {
    const RkGeo &geo = *geo_p;
    const int net = blockIdx.x / geo.n_sites, s = blockIdx.x % geo.n_sites;
    const double *t = T_all + (size_t)net * net_stride + geo.toff[s];
    double *P = P_all + ((size_t)net * geo.n_sites + s) * (size_t)(CHI * CHI * CHI * CHI);
    const int rk = geo.rank[s];
    int slot[4];
    for (int d = 0; d < 4; ++d) slot[d] = geo.dir_slot[s][d];
    for (int e = threadIdx.x; e < CHI * CHI * CHI * CHI; e += kLt) {
        const int kk = e / (CHI * CHI), nn = e % (CHI * CHI);
        const int dig[4] = {kk / CHI, nn / CHI, kk % CHI, nn % CHI};  // -x, +x, -y, +y
        bool ok = true;
        int idx = 0;
        for (int d = 0; d < 4; ++d)
            if (slot[d] < 0 && dig[d] != 0) ok = false;
        if (ok)
            for (int l = 0; l < rk; ++l) {
                int dg = 0;
                for (int d = 0; d < 4; ++d)
                    if (slot[d] == l) dg = dig[d];
                idx = idx * CHI + dg;
            }
        P[e] = ok ? gld(t + idx) : 0.0;
    }
}

// Every (network, term) pair: the lattice contracted row-major with the
// term's diagonal operator on each bond (code 0: the weight S_b; 1: its first
// r entries (P); 2: the rest (Q)), applied to a site's +x and +y outputs.  The
// state [h][c_0]..[c_{Lx-1}] (chi^(Lx+1) doubles, two buffers per block in
// st_all) is rescaled at the end of each row, the log carried.  Each site is
// absorbed as C[o][n] = sum_k A[o][k] P_s[k][n] on the FP64 matrix cores:
// o = the other columns' indices, k = (h, c_x), n = (h', c'_x); a wave owns
// 16 x 64 output blocks (four 16 x 16 tiles sharing the A fragment).
template <int CHI>
__global__ void __launch_bounds__(kLt) k_terms_mfma(const RkGeo *__restrict__ geo_p, const double *__restrict__ P_all,
                                                      const double *__restrict__ S_all, const int8_t *__restrict__ ops,
                                                      int n_terms, int n_items, int r, double *__restrict__ st_all,
                                                      double *__restrict__ out) {
    const RkGeo &geo = *geo_p;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int Lx = geo.Lx;
    constexpr int KD = CHI * CHI;  // k and n ranges
    int NS = CHI;
    for (int x = 0; x < Lx; ++x) NS *= CHI;
    const int O = NS / KD;  // chi^(Lx-1)
    double *st0 = st_all + (size_t)blockIdx.x * 2 * NS;
    double *st1 = st0 + NS;
    __shared__ double dR[CHI], dD[CHI], red[4];
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
        const int net = item / n_terms, term = item % n_terms;
        const double *Sn = S_all + (size_t)net * kRkBonds * kRkLargeChi;
        const int8_t *op = ops + (size_t)term * geo.n_bonds;
        for (int e = tid; e < NS; e += kLt) st0[e] = e == 0 ? 1.0 : 0.0;
        double *cur = st0, *nxt = st1;
        double log_acc = 0.0;
        __syncthreads();
        for (int y = 0; y < geo.Ly; ++y) {
            for (int x = 0; x < Lx; ++x) {
                const int s = x + Lx * y;
                if (tid < CHI) {
                    for (int k = 0; k < 2; ++k) {
                        const int sl = geo.dir_slot[s][k == 0 ? 1 : 3];
                        double d = tid == 0 ? 1.0 : 0.0;
                        if (sl >= 0) {
                            const int b = geo.leg_bond[s][sl];
                            const int code = op[b];
                            d = Sn[b * kRkLargeChi + tid];
                            if ((code == 1 && tid >= r) || (code == 2 && tid < r)) d = 0.0;
                        }
                        (k == 0 ? dR : dD)[tid] = d;
                    }
                }
                __syncthreads();
                const bool has_l = geo.dir_slot[s][0] >= 0, has_u = geo.dir_slot[s][2] >= 0;
                const bool has_r = geo.dir_slot[s][1] >= 0, has_d = geo.dir_slot[s][3] >= 0;
                const double *Ps = P_all + ((size_t)net * geo.n_sites + s) * (size_t)(KD * KD);
                int lo_n = 1;  // chi^(Lx-1-x): range of the columns after x
                for (int k = x + 1; k < Lx; ++k) lo_n *= CHI;
                const int hi_mul = lo_n * CHI;        // stride of the columns before x
                const int h_mul = NS / CHI;            // stride of h
                auto addr = [&](int o, int kk) {       // state index of (other columns o, (h, c_x) = kk)
                    const int hi = o / lo_n, lo = o - hi * lo_n;
                    return (kk / CHI) * h_mul + hi * hi_mul + (kk % CHI) * lo_n + lo;
                };
                const int ngroups = (O / 16) * (KD / 64);
                for (int gi = wave; gi < ngroups; gi += kLt / 64) {
                    const int ot = gi / (KD / 64), ntile = gi - ot * (KD / 64);
                    const int o0 = ot * 16, n0 = ntile * 64;
                    // output columns n = (h', c'): zero unless absent legs keep index 0
                    bool live = false;
                    for (int q = 0; q < 64 && !live; ++q) {
                        const int n = n0 + q;
                        live = (has_r || n / CHI == 0) && (has_d || n % CHI == 0);
                    }
                    double4_t acc[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) acc[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
                    if (live) {
                        for (int k0 = 0; k0 < KD; k0 += 4) {
                            // skip k-steps whose (h, c) rows are all structurally zero
                            bool kl = false;
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const int kk = k0 + q;
                                kl = kl || ((has_l || kk / CHI == 0) && (has_u || kk % CHI == 0));
                            }
                            if (!kl) continue;
                            const int kk = k0 + (lane >> 4);
                            const double av = cur[addr(o0 + (lane & 15), kk)];
                            const double *prow = Ps + (size_t)kk * KD + n0 + (lane & 15);
#pragma unroll
                            for (int t = 0; t < 4; ++t)
                                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, gld(prow + 16 * t), acc[t], 0, 0, 0);
                        }
                    }
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int n = n0 + 16 * t + (lane & 15);
                        const double sc = dR[n / CHI] * dD[n % CHI];
#pragma unroll
                        for (int i = 0; i < 4; ++i) nxt[addr(o0 + 4 * i + (lane >> 4), n)] = acc[t][i] * sc;
                    }
                }
                __syncthreads();
                double *tsw = cur;
                cur = nxt;
                nxt = tsw;
            }
            // rescale by the largest magnitude at the end of the row
            double mx = 0.0;
            for (int e = tid; e < NS; e += kLt) mx = fmax(mx, fabs(cur[e]));
            mx = block_max(mx, red);
            if (mx > 0.0) {
                for (int e = tid; e < NS; e += kLt) cur[e] /= mx;
                log_acc += log(mx);
            }
            __syncthreads();
        }
        if (tid == 0) {
            out[2 * (size_t)item] = log_acc;
            out[2 * (size_t)item + 1] = cur[0];
        }
        __syncthreads();
    }
}

// Gather the networks' site tensors into [net][packed sites] (geo.toff).
__global__ void k_gather_large(const double *const *__restrict__ src, const RkGeo *__restrict__ geo_p,
                               int64_t net_stride, double *__restrict__ T_all) {
    const RkGeo &geo = *geo_p;
    const int net = blockIdx.x;
    for (int s = 0; s < geo.n_sites; ++s) {
        const double *p = src[(size_t)net * geo.n_sites + s];
        const int size = geo.toff[s + 1] - geo.toff[s];
        for (int e = threadIdx.x; e < size; e += blockDim.x)
            T_all[(size_t)net * net_stride + geo.toff[s] + e] = gld(p + e);
    }
}

}  // namespace

bool rank_large_supported(int chi, int Lx, int Ly) {
    if (chi != 8 && chi != 16) return false;
    if (Lx < 2 || Ly < 1 || Lx * Ly > kRkSites) return false;
    long long o = 1, ns = chi;
    for (int x = 0; x < Lx; ++x) ns *= chi;
    for (int x = 0; x < Lx - 1; ++x) o *= chi;
    return o % 16 == 0 && ns <= 65536;
}

template <int CHI>
static void launch_large(hipStream_t s, int n, int n_sites, int n_items, int grid, const RkGeo *g, double *T,
                         int64_t net_stride, double *scr, int64_t scr_stride, double *Sw, double *Lg, int *Sp, int *St,
                         double *P, const int8_t *ops, int n_terms, int r, double *st, double *terms,
                         const pne_rank_options *opt, RankTimer &timer) {
    hipLaunchKernelGGL(k_wpl<CHI>, dim3(n), dim3(kLt), 0, s, g, T, net_stride, scr, scr_stride, Sw, Lg, Sp, St,
                       opt->alpha, opt->ramp_sweeps, opt->max_sweeps, opt->tol);
    timer.mark(s);
    hipLaunchKernelGGL(k_pad_sites<CHI>, dim3((unsigned)n * n_sites), dim3(kLt), 0, s, g, T, net_stride, P);
    timer.mark(s);
    hipLaunchKernelGGL(k_terms_mfma<CHI>, dim3(grid), dim3(kLt), 0, s, g, P, Sw, ops, n_terms, n_items, r, st, terms);
    timer.mark(s);
}

pne_status rank_expand_large(pne_ctx *ctx, pne_network *const *nets, int32_t n, const RkGeo &geo,
                             const std::vector<int8_t> &ops, const std::vector<int8_t> &sgn, int n_terms,
                             const pne_rank_options *opt, pne_rank_result *results, RankTimer &timer) {
    const int chi = geo.chi, n_sites = geo.n_sites;
    const int64_t net_stride = ((int64_t)geo.toff[n_sites] + 31) & ~int64_t(31);
    const int64_t chi4 = (int64_t)chi * chi * chi * chi;
    const int64_t scr_stride = 3 * chi4;
    int64_t ns = chi;
    for (int x = 0; x < geo.Lx; ++x) ns *= chi;
    const int n_items = n * n_terms;
    const int grid = n_items < 512 ? n_items : 512;  // blocks of the term kernel (two state buffers each)
    hipStream_t s = ctx_stream(ctx);
    std::vector<const double *> src((size_t)n * n_sites);
    for (int i = 0; i < n; ++i)
        for (int q = 0; q < n_sites; ++q) src[(size_t)i * n_sites + q] = network_site_ptr(nets[i], q);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t oGeo = take(sizeof(RkGeo)), oSrc = take(src.size() * sizeof(double *)),
                 oT = take((size_t)n * net_stride * 8), oScr = take((size_t)n * scr_stride * 8),
                 oS = take((size_t)n * kRkBonds * kRkLargeChi * 8), oLog = take((size_t)n * 8),
                 oSw = take((size_t)n * 4), oSt = take((size_t)n * 4), oOps = take(ops.size()),
                 oSgn = take(sgn.size()), oP = take((size_t)n * n_sites * chi4 * 8),
                 oState = take((size_t)grid * 2 * ns * 8), oTerms = take((size_t)n_items * 2 * 8),
                 oRes = take((size_t)n * sizeof(pne_rank_result));
    void *buf = nullptr;
    if (hipMalloc(&buf, off) != hipSuccess)
        return ctx_fail(ctx, PNE_ERR_OUT_OF_MEMORY, "rank expansion: hipMalloc failed");
    char *B = static_cast<char *>(buf);
    auto fin = [&](pne_status r) {
        (void)hipFree(buf);
        return r;
    };
#define RKL_TRY(expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fin(ctx_fail(ctx, PNE_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_))); \
    } while (0)
    RKL_TRY(hipMemcpyAsync(B + oGeo, &geo, sizeof geo, hipMemcpyHostToDevice, s));
    RKL_TRY(hipMemcpyAsync(B + oSrc, src.data(), src.size() * sizeof(double *), hipMemcpyHostToDevice, s));
    RKL_TRY(hipMemcpyAsync(B + oOps, ops.data(), ops.size(), hipMemcpyHostToDevice, s));
    RKL_TRY(hipMemcpyAsync(B + oSgn, sgn.data(), sgn.size(), hipMemcpyHostToDevice, s));
    auto *g = reinterpret_cast<const RkGeo *>(B + oGeo);
    auto *T = reinterpret_cast<double *>(B + oT);
    timer.mark(s);
    hipLaunchKernelGGL(k_gather_large, dim3(n), dim3(kLt), 0, s, reinterpret_cast<const double *const *>(B + oSrc), g,
                       net_stride, T);
    RKL_TRY(hipGetLastError());
    timer.mark(s);
    auto *scr = reinterpret_cast<double *>(B + oScr);
    auto *Sw = reinterpret_cast<double *>(B + oS);
    auto *Lg = reinterpret_cast<double *>(B + oLog);
    auto *Sp = reinterpret_cast<int *>(B + oSw);
    auto *St = reinterpret_cast<int *>(B + oSt);
    auto *P = reinterpret_cast<double *>(B + oP);
    auto *st = reinterpret_cast<double *>(B + oState);
    auto *terms = reinterpret_cast<double *>(B + oTerms);
    const auto *opd = reinterpret_cast<const int8_t *>(B + oOps);
    if (chi == 8)
        launch_large<8>(s, n, n_sites, n_items, grid, g, T, net_stride, scr, scr_stride, Sw, Lg, Sp, St, P, opd,
                        n_terms, opt->rank, st, terms, opt, timer);
    else
        launch_large<16>(s, n, n_sites, n_items, grid, g, T, net_stride, scr, scr_stride, Sw, Lg, Sp, St, P, opd,
                         n_terms, opt->rank, st, terms, opt, timer);
    RKL_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_rank_combine, dim3((n + 63) / 64), dim3(64), 0, s, terms,
                       reinterpret_cast<const int8_t *>(B + oSgn), n_terms, n, Lg,
                       reinterpret_cast<pne_rank_result *>(B + oRes), Sp, St);
    RKL_TRY(hipGetLastError());
    timer.mark(s);
    RKL_TRY(hipMemcpyAsync(results, B + oRes, (size_t)n * sizeof(pne_rank_result), hipMemcpyDeviceToHost, s));
    RKL_TRY(hipStreamSynchronize(s));
#undef RKL_TRY
    timer.read(ctx_rank_times(ctx), 5);
    pne_status stt = PNE_OK;
    for (int i = 0; i < n; ++i) {
        if (results[i].status < 0 && stt == PNE_OK) stt = (pne_status)results[i].status;
        else if (results[i].status > 0 && stt == PNE_OK) stt = (pne_status)results[i].status;
    }
    return fin(stt);
}

}  // namespace pne
