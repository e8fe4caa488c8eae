// Strip expansion of an infinite, translation-invariant square-lattice
// network (Sec. IV.C).  One tensor A[l, r, u, d] (legs -x, +x, -y, +y, bond
// dimension chi) repeats on every site.  The path:
//
//   1. uniform BP: the four messages arriving on a site's legs (k_uniform_bp);
//   2. for each width k = 1..L and each direction, the leading eigenvalue of
//      the width-k transfer matrix with its two outer legs capped by the
//      arriving messages, by power iteration.  One application of the
//      transfer matrix is k streaming passes over a chi^k (or chi^(k+1))
//      vector, each applying one site as a (chi^2 x chi^2) matrix on the pair
//      (horizontal bond, one vertical index) (k_strip_pass).  The vertical
//      iteration starts from the product of the top caps, so its first L
//      applications also give the capped k x p patches (dot with the product
//      of the bottom caps, fused into the last pass);
//   3. the combinatorial sum (Eq. (7)) over the L vertical and L horizontal
//      strip partitions per unit cell (k_strip_combine).
//
// Every quantity is divided by the BP value per site raised to its number of
// sites, so the cell sums are O(1) at any L.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gmem.h"
#include "pne.h"
#include "runtime.h"

namespace pne {
namespace {

using dev::gld;
using dev::gst;

constexpr int kSt = 256;      // threads of the streaming passes and reductions
constexpr int kMaxChi = 6;
constexpr int kMaxL = 16;

// device scalars written by k_uniform_bp
enum { SC_NH = 0, SC_NV, SC_Z, SC_WBP, SC_FBP, SC_RES, SC_COUNT };

// Jacobi BP on the infinite lattice from uniform messages: each sweep
// computes all four messages from the previous ones, normalises them (L2,
// sign fixed so the entries sum to >= 0) and stops when no entry moved by
// more than tol, or after max_iter sweeps.  Then z (A with all four
// arriving messages), the bond overlaps n_h = mR.mL and n_v = mD.mU, and
// the BP value per site z / (n_h n_v).  msg = [mL | mR | mU | mD].
__global__ void __launch_bounds__(64) k_uniform_bp(const double *__restrict__ A, int chi, double tol, int max_iter,
                                                   double *__restrict__ msg, double *__restrict__ sc,
                                                   int *__restrict__ iters) {
    __shared__ double a[kMaxChi * kMaxChi * kMaxChi * kMaxChi];
    __shared__ double m[4][kMaxChi], nm[4][kMaxChi];
    __shared__ double red[4];
    __shared__ int done;
    const int t = threadIdx.x;
    const int c4 = chi * chi * chi * chi;
    for (int e = t; e < c4; e += 64) a[e] = A[e];
    if (t < 4 * chi) m[t / chi][t % chi] = 1.0 / sqrt((double)chi);
    if (t == 0) done = 0;
    __syncthreads();
    int it = 0;
    double res = 0.0;
    while (true) {
        if (t < 4 * chi) {
            const int dir = t / chi, o = t % chi;
            double s = 0.0;
            for (int x = 0; x < chi; ++x)
                for (int y = 0; y < chi; ++y)
                    for (int z = 0; z < chi; ++z) {
                        int l, r, u, d;
                        double w;
                        if (dir == 0) {  // arrives on -x: sent out of the left neighbour's +x
                            l = x, r = o, u = y, d = z;
                            w = m[0][l] * m[2][u] * m[3][d];
                        } else if (dir == 1) {  // arrives on +x
                            l = o, r = x, u = y, d = z;
                            w = m[1][r] * m[2][u] * m[3][d];
                        } else if (dir == 2) {  // arrives on -y
                            l = x, r = y, u = z, d = o;
                            w = m[0][l] * m[1][r] * m[2][u];
                        } else {  // arrives on +y
                            l = x, r = y, u = o, d = z;
                            w = m[0][l] * m[1][r] * m[3][d];
                        }
                        s = fma(a[((l * chi + r) * chi + u) * chi + d], w, s);
                    }
            nm[dir][o] = s;
        }
        __syncthreads();
        if (t < 4) {
            double nn = 0.0, sum = 0.0;
            for (int o = 0; o < chi; ++o) {
                nn = fma(nm[t][o], nm[t][o], nn);
                sum += nm[t][o];
            }
            const double inv = (sum < 0.0 ? -1.0 : 1.0) / sqrt(nn);
            double r = 0.0;
            for (int o = 0; o < chi; ++o) {
                nm[t][o] *= inv;
                r = fmax(r, fabs(nm[t][o] - m[t][o]));
            }
            red[t] = r;
        }
        __syncthreads();
        if (t < 4 * chi) m[t / chi][t % chi] = nm[t / chi][t % chi];
        ++it;
        if (t == 0) {
            res = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
            done = (res <= tol || it >= max_iter) ? 1 : 0;
        }
        __syncthreads();
        if (done) break;
        __syncthreads();
    }
    if (t < 4 * chi) msg[t] = m[t / chi][t % chi];
    if (t == 0) {
        double z = 0.0;
        for (int l = 0; l < chi; ++l)
            for (int r = 0; r < chi; ++r)
                for (int u = 0; u < chi; ++u)
                    for (int d = 0; d < chi; ++d)
                        z = fma(a[((l * chi + r) * chi + u) * chi + d], m[0][l] * m[1][r] * m[2][u] * m[3][d], z);
        double nh = 0.0, nv = 0.0;
        for (int o = 0; o < chi; ++o) {
            nh = fma(m[1][o], m[0][o], nh);
            nv = fma(m[3][o], m[2][o], nv);
        }
        const double w = z / (nh * nv);
        sc[SC_NH] = nh;
        sc[SC_NV] = nv;
        sc[SC_Z] = z;
        sc[SC_WBP] = w;
        sc[SC_FBP] = -log(w);
        sc[SC_RES] = res;
        *iters = it;
    }
}

// Site matrices of one direction (dir 0: vertical strips, a row of sites;
// dir 1: horizontal strips, the lattice with x and y exchanged, so the
// site's legs read (-y, +y, -x, +x) and the messages (mU, mD, mL, mR)).
// With A' the site in that reading and (cl, cr) the caps of its outer legs:
//   mid   [(h, i), (h', o)] = A'[h, h', i, o]
//   first [i, (h', o)]      = sum_l cl[l] A'[l, h', i, o]
//   last  [(h, i), o]       = sum_r A'[h, r, i, o] cr[r]
//   single[i, o]            = sum_{l, r} cl[l] A'[l, r, i, o] cr[r]
// followed by the top and bottom caps of the strip (the -y' and +y'
// arrivals).  Layout: mid chi^4 | first chi^3 | last chi^3 | single chi^2 |
// top chi | bottom chi.
__global__ void __launch_bounds__(kSt) k_strip_mats(const double *__restrict__ A, int chi,
                                                    const double *__restrict__ msg, int dir,
                                                    double *__restrict__ out) {
    const int c = chi, c2 = c * c, c3 = c2 * c, c4 = c3 * c;
    const double *cl = msg + (dir == 0 ? 0 : 2) * c;
    const double *cr = msg + (dir == 0 ? 1 : 3) * c;
    const double *top = msg + (dir == 0 ? 2 : 0) * c;
    const double *bot = msg + (dir == 0 ? 3 : 1) * c;
    auto at = [&](int l, int r, int i, int o) {
        // A'[l, r, i, o]: dir 1 reads A[i, o, l, r]
        return dir == 0 ? A[((l * c + r) * c + i) * c + o] : A[((i * c + o) * c + l) * c + r];
    };
    double *mid = out, *first = mid + c4, *last = first + c3, *single = last + c3, *tb = single + c2;
    for (int e = threadIdx.x; e < c4; e += kSt) {
        const int h = e / c3, i = (e / c2) % c, h2 = (e / c) % c, o = e % c;
        mid[(h * c + i) * c2 + h2 * c + o] = at(h, h2, i, o);
    }
    for (int e = threadIdx.x; e < c3; e += kSt) {
        const int i = e / c2, h2 = (e / c) % c, o = e % c;
        double s = 0.0;
        for (int l = 0; l < c; ++l) s = fma(cl[l], at(l, h2, i, o), s);
        first[i * c2 + h2 * c + o] = s;
        const int h = e / c2, i2 = (e / c) % c, o2 = e % c;
        double s2 = 0.0;
        for (int r = 0; r < c; ++r) s2 = fma(at(h, r, i2, o2), cr[r], s2);
        last[(h * c + i2) * c + o2] = s2;
    }
    for (int e = threadIdx.x; e < c2; e += kSt) {
        const int i = e / c, o = e % c;
        double s = 0.0;
        for (int l = 0; l < c; ++l)
            for (int r = 0; r < c; ++r) s = fma(cl[l] * cr[r], at(l, r, i, o), s);
        single[i * c + o] = s;
    }
    for (int e = threadIdx.x; e < c; e += kSt) {
        tb[e] = top[e];
        tb[c + e] = bot[e];
    }
}

// x[idx] = prod over the k base-chi digits of idx of v[digit].
__global__ void __launch_bounds__(kSt) k_fill_product(double *__restrict__ x, const double *__restrict__ v, int chi,
                                                      int k, int64_t n, double *__restrict__ scale) {
    const int64_t t = (int64_t)blockIdx.x * kSt + threadIdx.x;
    if (t == 0) *scale = 1.0;
    if (t >= n) return;
    int64_t r = t;
    double p = 1.0;
    for (int d = 0; d < k; ++d) {
        p *= v[r % chi];
        r /= chi;
    }
    x[t] = p;
}

// One site of a transfer-matrix application.  The input holds the indices
// [h][pre][i][post] (h absent when HI == 1), the output [h'][pre][o][post]
// (h' absent when HO == 1); each thread takes one (pre, post) pair and
// applies the (HI chi) x (HO chi) site matrix M.  Consecutive threads take
// consecutive post, so every load and store of a wave is contiguous when
// post >= 64.  HI == 1 (first site): the input is multiplied by *scale.
// LAST (HO == 1, post == 1): also the block's sums of x.y, y.y and b.y, x
// being the iteration's input vector and b the product of the bottom caps.
template <int CV, int HI, int HO, bool LAST>
__global__ void __launch_bounds__(kSt) k_strip_pass(const double *__restrict__ X, double *__restrict__ Y,
                                                    const double *__restrict__ M, int64_t pre, int64_t post,
                                                    const double *__restrict__ scale, const double *__restrict__ Xo,
                                                    const double *__restrict__ bv, int pre_digits,
                                                    double *__restrict__ partials) {
    __shared__ double m[HI * CV * HO * CV];
    __shared__ double red[3][kSt / 64];
    for (int e = threadIdx.x; e < HI * CV * HO * CV; e += kSt) m[e] = M[e];
    __syncthreads();
    const int64_t n = pre * post;
    const int64_t t = (int64_t)blockIdx.x * kSt + threadIdx.x;
    double sxy = 0.0, syy = 0.0, sby = 0.0;
    if (t < n) {
        const int64_t p = t / post, q = t - p * post;
        double in[HI * CV];
        const double s = HI == 1 ? gld(scale) : 1.0;
#pragma unroll
        for (int h = 0; h < HI; ++h)
#pragma unroll
            for (int i = 0; i < CV; ++i) in[h * CV + i] = s * gld(&X[(((int64_t)h * pre + p) * CV + i) * post + q]);
        double bpre = 1.0;
        if (LAST) {
            int64_t r = p;
            for (int d = 0; d < pre_digits; ++d) {
                bpre *= bv[r % CV];
                r /= CV;
            }
        }
#pragma unroll
        for (int h = 0; h < HO; ++h)
#pragma unroll
            for (int o = 0; o < CV; ++o) {
                double acc = 0.0;
#pragma unroll
                for (int e = 0; e < HI * CV; ++e) acc = fma(m[e * (HO * CV) + h * CV + o], in[e], acc);
                const int64_t oi = (((int64_t)h * pre + p) * CV + o) * post + q;
                gst(&Y[oi], acc);
                if (LAST) {
                    const double x0 = gld(&Xo[oi]);
                    sxy = fma(x0, acc, sxy);
                    syy = fma(acc, acc, syy);
                    sby = fma(bpre * bv[o], acc, sby);
                }
            }
    }
    if (LAST) {
        for (int o = 32; o > 0; o >>= 1) {
            sxy += __shfl_xor(sxy, o, 64);
            syy += __shfl_xor(syy, o, 64);
            sby += __shfl_xor(sby, o, 64);
        }
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            red[0][w] = sxy;
            red[1][w] = syy;
            red[2][w] = sby;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            double v = 0.0;
            for (int k = 0; k < kSt / 64; ++k) v += red[threadIdx.x][k];
            partials[(int64_t)blockIdx.x * 3 + threadIdx.x] = v;
        }
    }
}

// Two neighbouring sites j, j+1 in one pass (chi <= 4): input
// [h][pre][i1][i2][post], output [h'][pre][o1][o2][post].  Site j maps
// (h, i1) -> (g, o1) for every i2 with M1 ((HI chi) x (chi chi)); site j+1
// maps (g, i2) -> (h', o2) for every o1 with M2 ((chi chi) x (HO chi)).
// A block takes 64 consecutive (pre, post) positions and stages their inputs
// in LDS; wave w then computes every output with o1 = w, so a thread keeps
// only one chi x chi slice of the intermediate.  Staging follows memory
// order: with post >= 64 a wave's 64 positions are 64 consecutive doubles
// for every input index; with post < 64 (the last sites of an application)
// the block's positions cover whole rows of post, so for each h its inputs
// are one contiguous run of 64 chi^2 doubles, copied as such, and the
// outputs are written back the same way through LDS.  Halves the passes over
// the vector; the rest as in k_strip_pass.
template <int CV, int HI, int HO, bool LAST, bool CONTIG>
__global__ void __launch_bounds__(64 * CV) k_strip_pass2(const double *__restrict__ X, double *__restrict__ Y,
                                                         const double *__restrict__ M1, const double *__restrict__ M2,
                                                         int64_t pre, int64_t post, int post_shift,
                                                         const double *__restrict__ scale,
                                                         const double *__restrict__ Xo,
                                                         const double *__restrict__ bv, int pre_digits,
                                                         double *__restrict__ partials) {
    constexpr int G = CV;                               // bond between the two sites
    constexpr int NT = 64 * CV;                         // threads
    constexpr int NV = HI * CV * CV;                    // inputs per position
    constexpr int NO = HO * CV * CV;                    // outputs per position
    constexpr int NB = (CONTIG && NO > NV) ? NO : NV;
    constexpr int RUN = 64 * CV * CV;                   // contiguous run per bond index h
    __shared__ double buf[NB][64];
    __shared__ double bq[CONTIG && LAST ? 64 : 1];      // bottom-cap product per local row
    __shared__ double red[3][CV];
    const int tid = threadIdx.x, pos = tid & 63;
    // the wave's o1 is uniform, so the site matrices are read with scalar
    // loads straight from global memory (no LDS traffic for them)
    const int o1 = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t n = pre * post;
    const int64_t t0 = (int64_t)blockIdx.x * 64;
    const int64_t t = t0 + pos;
    const double s = HI == 1 ? gld(scale) : 1.0;
    // CONTIG (post = 2^post_shift < 64, n a multiple of 64): the block holds
    // whole rows p0 .. p0 + 64/post - 1, and for each h its inputs are the run
    // ((pl * CV + i1) * CV + i2) * post + q at (h pre + p0) CV^2 post.
    const int64_t p0 = t0 >> post_shift;
    const int pmask = (1 << post_shift) - 1;
    if (CONTIG) {
        for (int e = tid; e < HI * RUN; e += NT) {
            const int h = e / RUN, r = e - h * RUN;
            const int q = r & pmask, rest = r >> post_shift;
            const int i2 = rest % CV, i1 = (rest / CV) % CV, pl = rest / (CV * CV);
            buf[(h * CV + i1) * CV + i2][(pl << post_shift) + q] =
                s * gld(&X[((int64_t)h * pre + p0) * (CV * CV) * post + r]);
        }
        if (LAST && tid < (64 >> post_shift)) {
            int64_t r = p0 + tid;
            double b = 1.0;
            for (int d = 0; d < pre_digits; ++d) {
                b *= bv[r % CV];
                r /= CV;
            }
            bq[tid] = b;
        }
    } else if (t < n) {
        // input (h, i1, i2) of position (p, q) sits at p CV^2 post + q +
        // h pre CV^2 post + (i1 CV + i2) post
        const int64_t p = t / post, q = t - p * post;
        const double *xp = X + p * (CV * CV) * post + q;
        const int64_t hs = pre * (CV * CV) * post;
        for (int v = o1; v < NV; v += CV) {
            const int h = v / (CV * CV), c = v % (CV * CV);
            buf[v][pos] = s * gld(xp + h * hs + c * post);
        }
    }
    __syncthreads();
    double sxy = 0.0, syy = 0.0, sby = 0.0;
    if (t < n) {
        // mid[g][i2] = sum_{h, i1} M1[(h, i1), (g, o1)] x[(h, i1, i2)]; each
        // staged input is read from LDS once
        double mid[G][CV];
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int i2 = 0; i2 < CV; ++i2) mid[g][i2] = 0.0;
#pragma unroll 4
        for (int e = 0; e < HI * CV; ++e)
#pragma unroll
            for (int i2 = 0; i2 < CV; ++i2) {
                const double x = buf[e * CV + i2][pos];
#pragma unroll
                for (int g = 0; g < G; ++g) mid[g][i2] = fma(M1[e * (G * CV) + g * CV + o1], x, mid[g][i2]);
            }
        double bpre = 1.0;
        int64_t p = 0, q = 0;
        double *yp = Y;
        const double *xop = Xo;
        if (!CONTIG) {
            p = t / post;
            q = t - p * post;
            // output (h', o1, o2) at p CV^2 post + q + h' pre CV^2 post + (o1 CV + o2) post
            yp = Y + p * (CV * CV) * post + q + (int64_t)(o1 * CV) * post;
            if (LAST) xop = Xo + p * (CV * CV) * post + q + (int64_t)(o1 * CV) * post;
            if (LAST) {
                int64_t r = p;
                for (int d = 0; d < pre_digits; ++d) {
                    bpre *= bv[r % CV];
                    r /= CV;
                }
            }
        }
        double out[CONTIG ? HO : 1][CV];
        // y[(h', o1, o2)] = sum_{g, i2} m2[(g, i2), (h', o2)] mid[g][i2]
#pragma unroll
        for (int h = 0; h < HO; ++h)
#pragma unroll
            for (int o2 = 0; o2 < CV; ++o2) {
                double acc = 0.0;
#pragma unroll
                for (int g = 0; g < G; ++g)
#pragma unroll
                    for (int i2 = 0; i2 < CV; ++i2)
                        acc = fma(M2[(g * CV + i2) * (HO * CV) + h * CV + o2], mid[g][i2], acc);
                if (CONTIG) {
                    out[CONTIG ? h : 0][o2] = acc;
                } else {
                    const int64_t oi = (int64_t)h * pre * (CV * CV) * post + o2 * post;
                    gst(yp + oi, acc);
                    if (LAST) {
                        const double x0 = gld(xop + oi);
                        sxy = fma(x0, acc, sxy);
                        syy = fma(acc, acc, syy);
                        sby = fma(bpre * bv[o1] * bv[o2], acc, sby);
                    }
                }
            }
        if (CONTIG) {
            __syncthreads();  // every read of the staged inputs is done (all positions are < n here)
#pragma unroll
            for (int h = 0; h < HO; ++h)
#pragma unroll
                for (int o2 = 0; o2 < CV; ++o2) buf[(h * CV + o1) * CV + o2][pos] = out[CONTIG ? h : 0][o2];
        }
    }
    if (CONTIG) {
        __syncthreads();
        for (int e = tid; e < HO * RUN; e += NT) {
            const int h = e / RUN, r = e - h * RUN;
            const int q = r & pmask, rest = r >> post_shift;
            const int c2 = rest % CV, c1 = (rest / CV) % CV, pl = rest / (CV * CV);
            const double y = buf[(h * CV + c1) * CV + c2][(pl << post_shift) + q];
            const int64_t oi = ((int64_t)h * pre + p0) * (CV * CV) * post + r;
            gst(&Y[oi], y);
            if (LAST) {
                const double x0 = gld(&Xo[oi]);
                sxy = fma(x0, y, sxy);
                syy = fma(y, y, syy);
                sby = fma(bq[CONTIG && LAST ? pl : 0] * bv[c1] * bv[c2], y, sby);
            }
        }
    }
    if (LAST) {
        for (int o = 32; o > 0; o >>= 1) {
            sxy += __shfl_xor(sxy, o, 64);
            syy += __shfl_xor(syy, o, 64);
            sby += __shfl_xor(sby, o, 64);
        }
        if (pos == 0) {
            red[0][o1] = sxy;
            red[1][o1] = syy;
            red[2][o1] = sby;
        }
        __syncthreads();
        if (tid < 3) {
            double v = 0.0;
            for (int k = 0; k < CV; ++k) v += red[tid][k];
            partials[(int64_t)blockIdx.x * 3 + tid] = v;
        }
    }
}

// Sum of the last pass's block sums in a fixed order; hist[4 it ..] =
// (x.y, y.y, b.y, scale applied this iteration); the next scale is 1/|y|.
__global__ void __launch_bounds__(kSt) k_strip_reduce(const double *__restrict__ partials, int64_t nblocks,
                                                      double *__restrict__ hist, int it, double *__restrict__ scale) {
    __shared__ double red[3][kSt / 64];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int64_t i = threadIdx.x; i < nblocks; i += kSt) {
        a += partials[3 * i];
        b += partials[3 * i + 1];
        c += partials[3 * i + 2];
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = a;
        red[1][w] = b;
        red[2][w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int k = 0; k < kSt / 64; ++k) {
            s0 += red[0][k];
            s1 += red[1][k];
            s2 += red[2][k];
        }
        const double s = *scale;
        hist[4 * it] = s0;
        hist[4 * it + 1] = s1;
        hist[4 * it + 2] = s2;
        hist[4 * it + 3] = s;
        *scale = 1.0 / sqrt(s1);
    }
}

// Per-width results from one direction's iteration history: the leading
// eigenvalue s_n (x_n . y_n) of the last step, divided by the cut bond's
// overlap and by w_bp^k; for the vertical direction also the capped k x p
// patches, p = 1..L: (b . y_p) times the norms of the earlier steps, divided
// by n_v^k n_h^p w_bp^(k p).
__global__ void k_strip_finish(const double *__restrict__ hist, int n_it, int k, int L, int dir,
                               const double *__restrict__ sc, double *__restrict__ lam_out,
                               double *__restrict__ patch_row) {
    if (threadIdx.x != 0) return;
    const double nh = sc[SC_NH], nv = sc[SC_NV], w = sc[SC_WBP];
    const int last = n_it - 1;
    const double lam = hist[4 * last + 3] * hist[4 * last];
    *lam_out = lam / ((dir == 0 ? nh : nv) * pow(w, (double)k));
    if (!patch_row) return;
    double log_acc = 0.0;
    for (int p = 1; p <= L; ++p) {
        const int it = p - 1;
        const double by = hist[4 * it + 2];
        double sign = by < 0.0 ? -1.0 : 1.0;
        if (nv < 0.0 && (k & 1)) sign = -sign;
        if (nh < 0.0 && (p & 1)) sign = -sign;
        if (w < 0.0 && ((k * p) & 1)) sign = -sign;
        const double lz = log(fabs(by)) + log_acc - k * log(fabs(nv)) - p * log(fabs(nh)) -
                          (double)k * p * log(fabs(w));
        patch_row[p - 1] = by == 0.0 ? 0.0 : sign * exp(lz);
        log_acc += 0.5 * log(hist[4 * it + 1]);
    }
}

// sum over non-empty subsets x of the L cyclic offsets of
// (-1)^(|x|+1) prod_{gaps g of x} c[g], with d = -c and a[n] the sum over
// compositions of n of prod d: the sum is -sum_g g d[g] a[L - g] (the first
// gap is the one that covers offset 0, in g positions).
__device__ double cyclic_sum(const double *c, int L) {
    double a[kMaxL + 1];
    a[0] = 1.0;
    for (int n = 1; n <= L; ++n) {
        double s = 0.0;
        for (int g = 1; g <= n; ++g) s = fma(-c[g], a[n - g], s);
        a[n] = s;
    }
    double t = 0.0;
    for (int g = 1; g <= L; ++g) t = fma((double)g * -c[g], a[L - g], t);
    return -t;
}

// The per-cell sum of Eq. (7) over the strip partitions, and f.  Vertical
// strips only (two_d == 0): S = cyclic_sum(lam).  Both directions: the
// subsets with only vertical (only horizontal) partitions give
// cyclic_sum(lam^L) (cyclic_sum(gam^L)); a non-empty horizontal subset xh
// with any non-empty vertical subset gives (-1)^|xh| cyclic_sum(c) with
// c[g] = prod_{gaps h of xh} patch[g][h].  f = f_bp - ln(S) / (sites per cell).
__global__ void __launch_bounds__(kSt) k_strip_combine(const double *__restrict__ lam, const double *__restrict__ gam,
                                                       const double *__restrict__ patch, int L, int two_d,
                                                       const double *__restrict__ sc, double *__restrict__ out) {
    __shared__ double red[kSt / 64];
    double acc = 0.0;
    double c[kMaxL + 1];
    if (two_d) {
        const int nsub = 1 << L;
        for (int xh = 1 + threadIdx.x; xh < nsub; xh += kSt) {
            int gl[kMaxL], m = 0, first = -1, prev = -1;
            for (int b = 0; b < L; ++b)
                if (xh >> b & 1) {
                    if (prev >= 0) gl[m++] = b - prev;
                    else first = b;
                    prev = b;
                }
            gl[m++] = first + L - prev;
            for (int g = 1; g <= L; ++g) {
                double v = 1.0;
                for (int j = 0; j < m; ++j) v *= patch[(g - 1) * L + gl[j] - 1];
                c[g] = v;
            }
            acc += ((m & 1) ? -1.0 : 1.0) * cyclic_sum(c, L);
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double S = 0.0;
    for (int k = 0; k < kSt / 64; ++k) S += red[k];
    for (int g = 1; g <= L; ++g) c[g] = two_d ? pow(lam[g - 1], (double)L) : lam[g - 1];
    S += cyclic_sum(c, L);
    if (two_d) {
        for (int g = 1; g <= L; ++g) c[g] = pow(gam[g - 1], (double)L);
        S += cyclic_sum(c, L);
    }
    out[0] = S;
    out[1] = sc[SC_FBP] - log(S) / (two_d ? (double)L * L : (double)L);
}

template <int CV>
hipError_t launch_pass(int variant, const double *X, double *Y, const double *M, int64_t pre, int64_t post,
                       const double *scale, const double *Xo, const double *bv, int pre_digits, double *partials,
                       hipStream_t s) {
    const int64_t n = pre * post;
    const dim3 grid((unsigned)((n + kSt - 1) / kSt));
    switch (variant) {
        case 0:  // first
            hipLaunchKernelGGL((k_strip_pass<CV, 1, CV, false>), grid, dim3(kSt), 0, s, X, Y, M, pre, post, scale,
                               Xo, bv, pre_digits, partials);
            break;
        case 1:  // middle
            hipLaunchKernelGGL((k_strip_pass<CV, CV, CV, false>), grid, dim3(kSt), 0, s, X, Y, M, pre, post, scale,
                               Xo, bv, pre_digits, partials);
            break;
        case 2:  // last
            hipLaunchKernelGGL((k_strip_pass<CV, CV, 1, true>), grid, dim3(kSt), 0, s, X, Y, M, pre, post, scale,
                               Xo, bv, pre_digits, partials);
            break;
        default:  // single site (k = 1)
            hipLaunchKernelGGL((k_strip_pass<CV, 1, 1, true>), grid, dim3(kSt), 0, s, X, Y, M, pre, post, scale,
                               Xo, bv, pre_digits, partials);
            break;
    }
    return hipGetLastError();
}

template <int CV, bool CONTIG>
hipError_t launch_pair_c(int variant, const double *X, double *Y, const double *M1, const double *M2, int64_t pre,
                         int64_t post, int post_shift, const double *scale, const double *Xo, const double *bv,
                         int pre_digits, double *partials, hipStream_t s) {
    const int64_t n = pre * post;
    const dim3 grid((unsigned)((n + 63) / 64)), block(64 * CV);
    switch (variant) {
        case 0:  // first two sites
            hipLaunchKernelGGL((k_strip_pass2<CV, 1, CV, false, CONTIG>), grid, block, 0, s, X, Y, M1, M2, pre, post,
                               post_shift, scale, Xo, bv, pre_digits, partials);
            break;
        case 1:  // two middle sites
            hipLaunchKernelGGL((k_strip_pass2<CV, CV, CV, false, CONTIG>), grid, block, 0, s, X, Y, M1, M2, pre,
                               post, post_shift, scale, Xo, bv, pre_digits, partials);
            break;
        case 2:  // the last two sites
            hipLaunchKernelGGL((k_strip_pass2<CV, CV, 1, true, CONTIG>), grid, block, 0, s, X, Y, M1, M2, pre, post,
                               post_shift, scale, Xo, bv, pre_digits, partials);
            break;
        default:  // both sites of a width-2 strip
            hipLaunchKernelGGL((k_strip_pass2<CV, 1, 1, true, CONTIG>), grid, block, 0, s, X, Y, M1, M2, pre, post,
                               post_shift, scale, Xo, bv, pre_digits, partials);
            break;
    }
    return hipGetLastError();
}

// Whole rows of post in every block of 64 positions: post a power of two
// below 64 and the position count a multiple of 64.
template <int CV>
hipError_t launch_pair(int variant, const double *X, double *Y, const double *M1, const double *M2, int64_t pre,
                       int64_t post, const double *scale, const double *Xo, const double *bv, int pre_digits,
                       double *partials, hipStream_t s) {
    const int64_t n = pre * post;
    if (post < 64 && (post & (post - 1)) == 0 && n % 64 == 0) {
        int shift = 0;
        while ((int64_t(1) << shift) < post) ++shift;
        return launch_pair_c<CV, true>(variant, X, Y, M1, M2, pre, post, shift, scale, Xo, bv, pre_digits, partials,
                                       s);
    }
    return launch_pair_c<CV, false>(variant, X, Y, M1, M2, pre, post, 0, scale, Xo, bv, pre_digits, partials, s);
}

hipError_t pair(int chi, int variant, const double *X, double *Y, const double *M1, const double *M2, int64_t pre,
                int64_t post, const double *scale, const double *Xo, const double *bv, int pre_digits,
                double *partials, hipStream_t s) {
    switch (chi) {
        case 2: return launch_pair<2>(variant, X, Y, M1, M2, pre, post, scale, Xo, bv, pre_digits, partials, s);
        case 3: return launch_pair<3>(variant, X, Y, M1, M2, pre, post, scale, Xo, bv, pre_digits, partials, s);
        default: return launch_pair<4>(variant, X, Y, M1, M2, pre, post, scale, Xo, bv, pre_digits, partials, s);
    }
}

hipError_t pass(int chi, int variant, const double *X, double *Y, const double *M, int64_t pre, int64_t post,
                const double *scale, const double *Xo, const double *bv, int pre_digits, double *partials,
                hipStream_t s) {
    switch (chi) {
        case 2: return launch_pass<2>(variant, X, Y, M, pre, post, scale, Xo, bv, pre_digits, partials, s);
        case 3: return launch_pass<3>(variant, X, Y, M, pre, post, scale, Xo, bv, pre_digits, partials, s);
        case 4: return launch_pass<4>(variant, X, Y, M, pre, post, scale, Xo, bv, pre_digits, partials, s);
        case 5: return launch_pass<5>(variant, X, Y, M, pre, post, scale, Xo, bv, pre_digits, partials, s);
        default: return launch_pass<6>(variant, X, Y, M, pre, post, scale, Xo, bv, pre_digits, partials, s);
    }
}

int64_t ipow(int64_t b, int e) {
    int64_t r = 1;
    while (e-- > 0) r *= b;
    return r;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace
}  // namespace pne

using namespace pne;

extern "C" pne_status pne_strip_options_default(pne_strip_options *opt) {
    if (!opt) return PNE_ERR_INVALID_ARG;
    std::memset(opt, 0, sizeof *opt);
    opt->L = 2;
    opt->two_d = 1;
    opt->bp_tol = 1e-14;
    opt->bp_max_iter = 10000;
    opt->power_tol = 1e-13;
    opt->power_max_iter = 20000;
    opt->check_every = 4;
    return PNE_OK;
}

extern "C" pne_status pne_strip_expand(pne_ctx *ctx, const double *A, int32_t chi, const pne_strip_options *opt,
                                       pne_strip_result *res) {
    if (!ctx || !A || !opt || !res) return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "null argument");
    const int L = opt->L;
    if (chi < 2 || chi > kMaxChi) return ctx_fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: chi must be in [2, 6]");
    if (L < 1 || L > kMaxL) return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "L must be in [1, 16]");
    if (opt->power_max_iter < L || opt->bp_max_iter < 1 || opt->check_every < 1)
        return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "iteration caps too small (power_max_iter >= L)");
    const int64_t big = ipow(chi, L + 1);
    if (big > (int64_t(1) << 28)) return ctx_fail(ctx, PNE_ERR_UNSUPPORTED, "unsupported: chi^(L+1) above 2^28");
    for (int64_t e = 0; e < ipow(chi, 4); ++e)
        if (!std::isfinite(A[e])) return ctx_fail(ctx, PNE_ERR_INVALID_ARG, "tensor entry not finite");
    hipStream_t s = ctx_stream(ctx);
    const int c4 = chi * chi * chi * chi;
    const int mats = c4 + 2 * chi * chi * chi + chi * chi + 2 * chi;
    const int64_t vec = ipow(chi, L);
    const int64_t nblk_max = std::max((ipow(chi, L - 1) + kSt - 1) / kSt, (ipow(chi, std::max(L - 2, 0)) + 63) / 64);
    const int hist_n = 4 * opt->power_max_iter;
    // one allocation: A, msg, scalars, mats x2, out lam/gam/patch, combine out, scale, hist, partials,
    // x, y, t0, t1
    size_t off = 0;
    auto take = [&](size_t n) {
        size_t o = off;
        off += (n * sizeof(double) + 255) & ~size_t(255);
        return o;
    };
    const size_t oA = take(c4), oMsg = take(4 * chi), oSc = take(SC_COUNT + 2), oMats = take(2 * (size_t)mats),
                 oLam = take(L), oGam = take(L), oPatch = take((size_t)L * L), oOut = take(2), oScale = take(1),
                 oHist = take(hist_n), oPart = take(3 * (size_t)nblk_max), oX = take(vec), oY = take(vec),
                 oT0 = take(big), oT1 = take(big);
    DevBuf buf;
    hipError_t e = hipMalloc(&buf.p, off);
    if (e != hipSuccess) return ctx_fail(ctx, PNE_ERR_OUT_OF_MEMORY, "strip buffers: hipMalloc failed");
    char *base = static_cast<char *>(buf.p);
    auto D = [&](size_t o) { return reinterpret_cast<double *>(base + o); };
    int *d_iters = reinterpret_cast<int *>(D(oSc) + SC_COUNT);
    std::vector<double> h_hist(hist_n);
    res->reserved = 0;
    res->status = PNE_OK;
    res->power_iters = 0;
    res->n_unconverged = 0;

#define ST_TRY(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return ctx_fail(ctx, PNE_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

    ST_TRY(hipMemcpyAsync(D(oA), A, c4 * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_uniform_bp, dim3(1), dim3(64), 0, s, D(oA), chi, opt->bp_tol, opt->bp_max_iter, D(oMsg),
                       D(oSc), d_iters);
    ST_TRY(hipGetLastError());
    for (int dir = 0; dir < 2; ++dir) {
        hipLaunchKernelGGL(k_strip_mats, dim3(1), dim3(kSt), 0, s, D(oA), chi, D(oMsg), dir, D(oMats) + dir * mats);
        ST_TRY(hipGetLastError());
    }
    double h_sc[SC_COUNT + 2];
    ST_TRY(hipMemcpyAsync(h_sc, D(oSc), sizeof h_sc, hipMemcpyDeviceToHost, s));
    ST_TRY(hipStreamSynchronize(s));
    int bp_iters = 0;
    std::memcpy(&bp_iters, &h_sc[SC_COUNT], sizeof(int));
    res->bp_iters = bp_iters;
    res->bp_residual = h_sc[SC_RES];
    res->f_bp = h_sc[SC_FBP];
    if (!(h_sc[SC_WBP] > 0.0) || !std::isfinite(h_sc[SC_WBP]) || h_sc[SC_NH] == 0.0 || h_sc[SC_NV] == 0.0)
        return ctx_fail(ctx, PNE_ERR_SINGULAR, "BP value per site not positive, or a zero bond overlap");
    if (h_sc[SC_RES] > opt->bp_tol) res->status = PNE_WARN_BP_NOT_CONVERGED;

    const int ndir = opt->two_d ? 2 : 1;
    for (int dir = 0; dir < ndir; ++dir) {
        const double *M = D(oMats) + dir * mats;
        const double *Mmid = M, *Mfirst = M + c4, *Mlast = Mfirst + chi * chi * chi,
                     *Msingle = Mlast + chi * chi * chi, *top = Msingle + chi * chi, *bot = top + chi;
        for (int k = 1; k <= L; ++k) {
            double *x = D(oX), *y = D(oY);
            const int64_t nk = ipow(chi, k);
            hipLaunchKernelGGL(k_fill_product, dim3((unsigned)((nk + kSt - 1) / kSt)), dim3(kSt), 0, s, x, top, chi, k,
                               nk, D(oScale));
            ST_TRY(hipGetLastError());
            // the last pass runs one thread per chi^2 outputs (a pair) or chi (one site)
            const bool paired = chi <= 4 && !opt->single_site_passes;
            // the last pass is a pair (64 positions per block) when k is even
            const bool last_pair = paired && k >= 2 && k % 2 == 0;
            const int64_t nblk = k == 1 ? 1
                                 : last_pair ? (ipow(chi, k - 2) + 63) / 64
                                             : (ipow(chi, k - 1) + kSt - 1) / kSt;
            const int min_it = (dir == 0 && opt->two_d) ? L : 2;
            int it = 0, n_done = 0;
            bool conv = false;
            while (it < opt->power_max_iter && !conv) {
                if (k == 1) {
                    ST_TRY(pass(chi, 3, x, y, Msingle, 1, 1, D(oScale), x, bot, 0, D(oPart), s));
                } else if (paired && k == 2) {
                    ST_TRY(pair(chi, 3, x, y, Mfirst, Mlast, 1, 1, D(oScale), x, bot, 0, D(oPart), s));
                } else if (paired) {
                    // sites (1, 2) from x, then pairs (j, j + 1); the last one or two sites write y
                    double *t0 = D(oT0), *t1 = D(oT1);
                    ST_TRY(pair(chi, 0, x, t0, Mfirst, Mmid, 1, ipow(chi, k - 2), D(oScale), nullptr, nullptr, 0,
                                nullptr, s));
                    int j = 3;  // next site to apply
                    while (k - j + 1 > 2) {
                        ST_TRY(pair(chi, 1, t0, t1, Mmid, Mmid, ipow(chi, j - 1), ipow(chi, k - j - 1), nullptr,
                                    nullptr, nullptr, 0, nullptr, s));
                        std::swap(t0, t1);
                        j += 2;
                    }
                    if (k - j + 1 == 2)
                        ST_TRY(pair(chi, 2, t0, y, Mmid, Mlast, ipow(chi, k - 2), 1, nullptr, x, bot, k - 2, D(oPart),
                                    s));
                    else
                        ST_TRY(pass(chi, 2, t0, y, Mlast, ipow(chi, k - 1), 1, nullptr, x, bot, k - 1, D(oPart), s));
                } else {
                    double *t0 = D(oT0), *t1 = D(oT1);
                    ST_TRY(pass(chi, 0, x, t0, Mfirst, 1, ipow(chi, k - 1), D(oScale), nullptr, nullptr, 0, nullptr,
                                s));
                    for (int j = 2; j < k; ++j) {
                        ST_TRY(pass(chi, 1, t0, t1, Mmid, ipow(chi, j - 1), ipow(chi, k - j), nullptr, nullptr,
                                    nullptr, 0, nullptr, s));
                        std::swap(t0, t1);
                    }
                    ST_TRY(pass(chi, 2, t0, y, Mlast, ipow(chi, k - 1), 1, nullptr, x, bot, k - 1, D(oPart), s));
                }
                hipLaunchKernelGGL(k_strip_reduce, dim3(1), dim3(kSt), 0, s, D(oPart), nblk, D(oHist), it, D(oScale));
                ST_TRY(hipGetLastError());
                std::swap(x, y);
                ++it;
                if (it >= min_it && (it % opt->check_every == 0 || it == opt->power_max_iter)) {
                    ST_TRY(hipMemcpyAsync(h_hist.data() + 4 * n_done, D(oHist) + 4 * n_done,
                                          4 * (size_t)(it - n_done) * sizeof(double), hipMemcpyDeviceToHost, s));
                    ST_TRY(hipStreamSynchronize(s));
                    n_done = it;
                    if (it >= 3) {
                        auto lam_at = [&](int i) { return h_hist[4 * i + 3] * h_hist[4 * i]; };
                        const double l0 = lam_at(it - 1), l1 = lam_at(it - 2), l2 = lam_at(it - 3);
                        conv = std::fabs(l0 - l1) <= opt->power_tol * std::fabs(l0) &&
                               std::fabs(l1 - l2) <= opt->power_tol * std::fabs(l1);
                    }
                }
            }
            res->power_iters += it;
            if (res->iters) res->iters[dir * L + (k - 1)] = it;
            if (!conv) {
                res->n_unconverged += 1;
                if (res->status == PNE_OK) res->status = PNE_WARN_BP_NOT_CONVERGED;
            }
            double *lam_out = (dir == 0 ? D(oLam) : D(oGam)) + (k - 1);
            double *patch_row = (dir == 0 && opt->two_d) ? D(oPatch) + (size_t)(k - 1) * L : nullptr;
            hipLaunchKernelGGL(k_strip_finish, dim3(1), dim3(64), 0, s, D(oHist), it, k, L, dir, D(oSc), lam_out,
                               patch_row);
            ST_TRY(hipGetLastError());
        }
    }
    hipLaunchKernelGGL(k_strip_combine, dim3(1), dim3(kSt), 0, s, D(oLam), D(oGam), D(oPatch), L, opt->two_d ? 1 : 0,
                       D(oSc), D(oOut));
    ST_TRY(hipGetLastError());
    double h_out[2];
    ST_TRY(hipMemcpyAsync(h_out, D(oOut), sizeof h_out, hipMemcpyDeviceToHost, s));
    if (res->lam) ST_TRY(hipMemcpyAsync(res->lam, D(oLam), L * sizeof(double), hipMemcpyDeviceToHost, s));
    if (res->gam && opt->two_d) ST_TRY(hipMemcpyAsync(res->gam, D(oGam), L * sizeof(double), hipMemcpyDeviceToHost, s));
    if (res->patch && opt->two_d)
        ST_TRY(hipMemcpyAsync(res->patch, D(oPatch), (size_t)L * L * sizeof(double), hipMemcpyDeviceToHost, s));
    ST_TRY(hipStreamSynchronize(s));
#undef ST_TRY
    res->cell_sum = h_out[0];
    res->f = h_out[1];
    if (!(h_out[0] > 0.0) || !std::isfinite(h_out[1]))
        return ctx_fail(ctx, PNE_ERR_SINGULAR, "strip expansion: cell sum not positive");
    return (pne_status)res->status;
}
