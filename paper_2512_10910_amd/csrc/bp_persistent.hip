// Persistent belief propagation: one block runs every sweep of one network
// (Sec. II.B fixed-point messages; open legs are not handled here).  A
// bipartite network runs the red-black schedule in one message buffer (see
// the kernel), any other network Jacobi sweeps in two.
//
// The network's two message buffers, its site table (tensor pointer, local
// message offsets) and the site order of its tiles are staged in LDS once.
// Sites are grouped by shape (all legs of dimension D, rank R).  Inside a
// group a tile is SPW consecutive sites of the group list, laid out exactly as
// on the per-launch register path: the last T legs index lanes through
// power-of-two bit-fields, the first R-T legs index values held in registers,
// and every outgoing message is an xor-butterfly sum inside a site's lane
// segment.  Each wavefront loads NT tiles before computing any of them, so a
// tile costs one global round trip for its tensor data; the block-wide
// residual after every sweep decides convergence without leaving the kernel.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"
#include "regauge.h"
#include "terms.h"

namespace pne {

namespace {

constexpr int kPThreads = 512;
constexpr int kPWaves = kPThreads / 64;
constexpr int kPSmallThreads = 128;
// tiles in flight per wavefront for a shape with nl register values per tile
__host__ __device__ constexpr int tiles_in_flight(int nl) { return nl <= 4 ? 2 : 1; }

extern __shared__ double p_lds[];

__device__ inline double wave_max_p(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

constexpr int ipw(int b, int e) { return e <= 0 ? 1 : b * ipw(b, e - 1); }

// LDS layout of one block, in doubles (pointers take one double each, ints
// are packed two per double).
struct PLayout {
    int b0, b1;      // message buffers
    int tptr;        // n_sites tensor pointers
    int moff;        // n_sites ints: local message offsets
    int dst;         // n_sites * kMaxRank ints: local destination offsets
    int list;        // n_sites ints: local site ids in group order
    int vside;       // n_sites ints: mask of slots where the site is the bond's second site
    int soff;        // n_sites int64: slice offsets
    int scr;         // per-wave scratch
};

__device__ inline const double *tptr_at(const PLayout &L, int s) {
    return reinterpret_cast<const double *const *>(p_lds + L.tptr)[s];
}
__device__ inline int int_at(int off_doubles, int i) { return reinterpret_cast<const int *>(p_lds + off_doubles)[i]; }

// NT tiles of a (D, R) group: chunk c covers group positions
// [c*NT*SPW, (c+1)*NT*SPW).  Returns the wavefront's residual.
template <int D, int R>
__device__ __attribute__((noinline)) double ptiles(const PLayout L, int gl_off, int n_in_group, int chunk, int mi,
                                                   int mo, int scr, int *bad) {
    constexpr int P = D <= 2 ? 2 : (D <= 4 ? 4 : 8);
    constexpr int B = P == 2 ? 1 : (P == 4 ? 2 : 3);
    constexpr int T = (6 / B) < R ? (6 / B) : R;
    constexpr int NLEG = R - T;
    constexpr int LS = 1 << (B * T);
    constexpr int SPW = 64 / LS;
    constexpr int NL = ipw(D, NLEG);
    constexpr int DT = ipw(D, T);
    constexpr int ND = R * D;
    constexpr int kNT = tiles_in_flight(NL);
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
    const int base_pos = chunk * kNT * SPW;
    double tv[kNT][NL];
    double mt[kNT][T];
    double ml[kNT][NLEG > 0 ? NLEG : 1][D];
    bool act[kNT];
#pragma unroll
    for (int k = 0; k < kNT; ++k) {
        const int pos = base_pos + k * SPW + slot;
        act[k] = inseg && pos < n_in_group;
        const int site = int_at(L.list, gl_off + (pos < n_in_group ? pos : 0));
        const double *tp = tptr_at(L, site);
        const int mb = mi + int_at(L.moff, site);
#pragma unroll
        for (int q = 0; q < NL; ++q) tv[k][q] = dev::gld(tp + q * DT + toff);  // in bounds on every lane
#pragma unroll
        for (int m = 0; m < T; ++m) mt[k][m] = p_lds[mb + (NLEG + m) * D + dig[m] % D];
#pragma unroll
        for (int j = 0; j < NLEG; ++j)
#pragma unroll
            for (int i = 0; i < D; ++i) ml[k][j][i] = p_lds[mb + j * D + i];
    }
    // normalisation item of this lane: (tile k, site j in the tile, leg l)

    double *out = p_lds + scr;  // [tile][site][R*D]
#pragma unroll
    for (int k = 0; k < kNT; ++k) {
        const int oslot = (k * SPW + slot) * ND;
        double A = 0.0;
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            double w = 1.0;
#pragma unroll
            for (int j = 0; j < NLEG; ++j) w *= ml[k][j][(q / ipw(D, NLEG - 1 - j)) % D];
            A = fma(tv[k][q], w, A);
        }
        if (!inseg) A = 0.0;  // lanes past the last digit add nothing to the segment sums
#pragma unroll
        for (int m = 0; m < T; ++m) {
            double pm = A;
#pragma unroll
            for (int m2 = 0; m2 < T; ++m2)
                if (m2 != m) pm *= mt[k][m2];
#pragma unroll
            for (int m2 = 0; m2 < T; ++m2) {
                if (m2 == m) continue;
#pragma unroll
                for (int bit = 0; bit < B; ++bit) pm += __shfl_xor(pm, 1 << (B * (T - 1 - m2) + bit), 64);
            }
            bool owner = act[k];
#pragma unroll
            for (int m2 = 0; m2 < T; ++m2)
                if (m2 != m) owner = owner && dig[m2] == 0;
            if (owner) out[oslot + (NLEG + m) * D + dig[m]] = pm;
        }
        if (NLEG > 0) {
            double qt = act[k] ? 1.0 : 0.0;
#pragma unroll
            for (int m = 0; m < T; ++m) qt *= mt[k][m];
#pragma unroll
            for (int j = 0; j < NLEG; ++j) {
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    double sv = 0.0;
#pragma unroll
                    for (int q = 0; q < NL; ++q) {
                        if ((q / ipw(D, NLEG - 1 - j)) % D != i) continue;
                        double w = 1.0;
#pragma unroll
                        for (int j2 = 0; j2 < NLEG; ++j2)
                            if (j2 != j) w *= ml[k][j2][(q / ipw(D, NLEG - 1 - j2)) % D];
                        sv = fma(tv[k][q], w, sv);
                    }
                    sv *= qt;
#pragma unroll
                    for (int bit = 0; bit < B * T; ++bit) sv += __shfl_xor(sv, 1 << bit, 64);
                    if (tb == 0 && base_pos + k * SPW + slot < n_in_group) out[oslot + j * D + i] = sv;
                }
            }
        }
    }
    wave_sync();
    // normalisation items: (tile k, site j in the tile, leg l)
    double res = 0.0;
    for (int n = lane; n < kNT * SPW * R; n += 64) {
        const int ik = n / (SPW * R);
        const int irem = n - ik * (SPW * R);
        const int ij = irem / R;
        const int il = irem - ij * R;
        const int ipos = base_pos + ik * SPW + ij;
        if (ipos >= n_in_group) continue;
        const int site = int_at(L.list, gl_off + ipos);
        const int idst = int_at(L.dst, site * kMaxRank + il);
        const double *raw = out + (ik * SPW + ij) * ND + il * D;
        double n2 = 0.0, sum = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            n2 = fma(raw[i], raw[i], n2);
            sum += raw[i];
        }
        const double nrm = sqrt(n2);
        if (!(nrm > 0.0) || !isfinite(nrm)) {
            *bad = 1;
            continue;
        }
        const double inv = (sum < 0.0 ? -1.0 : 1.0) / nrm;  // L2 norm, sign fixed so the sum is >= 0
        double d1 = 0.0, d2 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double v = raw[i] * inv;
            const double old = p_lds[mi + idst + i];
            d1 = fmax(d1, fabs(v - old));
            d2 = fmax(d2, fabs(v + old));
            p_lds[mo + idst + i] = v;
        }
        res = fmax(res, fmin(d1, d2));
    }
    res = wave_max_p(res);
    wave_sync();
    return res;
}

// ---------------------------------------------------------------------------
// DPP variant for D <= 4: only the last T = min(R, 2) legs index lanes, so a
// site's lane segment (P^T <= 16 lanes) lies inside one DPP row and every
// reduction is a data-parallel-primitive move on the VALU: the low field
// (last leg) with quad permutations, the high field (second-to-last leg,
// P = 4) with row rotations by 4 and 8, which keep the low bits.  The first
// R-T legs index NL = D^(R-T) values per lane.
// Every control used here is a full permutation of a row, so no lane reads
// outside it and the DPP "old" operand is never needed.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
constexpr int kDppXor1 = 0xB1;    // quad_perm [1,0,3,2]: lane ^ 1
constexpr int kDppXor2 = 0x4E;    // quad_perm [2,3,0,1]: lane ^ 2
constexpr int kDppXor3 = 0x1B;    // quad_perm [3,2,1,0]: lane ^ 3
constexpr int kDppRor4 = 0x124;   // row_ror:4
constexpr int kDppRor8 = 0x128;   // row_ror:8
constexpr int kDppMirror = 0x140;      // row_mirror: lane ^ 15 within the row
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror: lane ^ 7 within each half row

// Partner lane (lane ^ MASK inside a 16-lane row) for the masks 15, 7, 3, 1,
// which span the four lane bits of a row.
template <int MASK>
__device__ inline double dpp_xor(double v) {
    if constexpr (MASK == 15) return dpp_f64<kDppMirror>(v);
    else if constexpr (MASK == 7) return dpp_f64<kDppHalfMirror>(v);
    else if constexpr (MASK == 3) return dpp_f64<kDppXor3>(v);
    else return dpp_f64<kDppXor1>(v);
}

template <int S, int STAGE>
__device__ inline double seg_partner(double x) {
    if constexpr (S == 4) return STAGE == 0 ? dpp_xor<15>(x) : (STAGE == 1 ? dpp_xor<7>(x) : (STAGE == 2 ? dpp_xor<3>(x) : dpp_xor<1>(x)));
    else if constexpr (S == 2) return STAGE == 0 ? dpp_xor<3>(x) : dpp_xor<1>(x);
    else return dpp_xor<1>(x);
}

// Stages STAGE.. of a segment reduction (see seg_reduce_stream) on the first
// NC entries of v; compile-time sizes keep every index static.
template <int S, int STAGE, int NC, int N>
__device__ inline void seg_stages(double (&v)[N], int tb, int &elem, bool &writer) {
    if constexpr (STAGE < S) {
        const bool hi = (tb >> (S - 1 - STAGE)) & 1;
        if constexpr (NC > 1) {
            constexpr int h = NC / 2;
#pragma unroll
            for (int k = 0; k < h; ++k) {
                const double send = hi ? v[k] : v[k + h];
                const double keep = hi ? v[k + h] : v[k];
                v[k] = keep + seg_partner<S, STAGE>(send);
            }
            elem = elem * 2 + (hi ? 1 : 0);
            seg_stages<S, STAGE + 1, h, N>(v, tb, elem, writer);
        } else {
            v[0] += seg_partner<S, STAGE>(v[0]);
            writer = writer && !hi;
            seg_stages<S, STAGE + 1, 1, N>(v, tb, elem, writer);
        }
    }
}

// Sum N per-lane values (N a power of two) over a segment of LS lanes (2, 4
// or 16, inside one DPP row) by recursive halving.  At stage s a lane and its
// partner lane ^ mask (masks 15/7/3/1 from the segment's top bit down) keep
// complementary halves of their vectors and add the partner's copy of the
// half they keep; once one value is left, later stages add it to the
// partner's.  part(e) produces element e's per-lane value on the fly and the
// first stage consumes the pairs (e, e + N/2) as they are made, so at most
// N/2 values stay live.  Afterwards v[0..m-1] (m = N / LS when N > LS,
// else 1) hold the segment totals of elements elem*m .. elem*m+m-1, the same
// in every lane sharing the kept bits; `writer` marks one of them.
template <int LS, int N, typename Part>
__device__ inline void seg_reduce_stream(const Part &part, double (&v)[N], int tb, int &elem, bool &writer) {
    constexpr int S = LS == 16 ? 4 : (LS == 4 ? 2 : 1);
    elem = 0;
    writer = true;
    const bool hi = (tb >> (S - 1)) & 1;
    if constexpr (N > 1) {
        constexpr int h = N / 2;
#pragma unroll
        for (int k = 0; k < h; ++k) {
            const double a = part(k), b = part(k + h);
            const double send = hi ? a : b;
            const double keep = hi ? b : a;
            v[k] = keep + seg_partner<S, 0>(send);
        }
        elem = hi ? 1 : 0;
        seg_stages<S, 1, h, N>(v, tb, elem, writer);
    } else {
        v[0] = part(0);
        v[0] += seg_partner<S, 0>(v[0]);
        writer = !hi;
        seg_stages<S, 1, 1, N>(v, tb, elem, writer);
    }
}

template <int P>
__device__ inline double sum_low(double v) {  // over the last leg's digit
    v += dpp_f64<kDppXor1>(v);
    if (P == 4) v += dpp_f64<kDppXor2>(v);
    return v;
}
template <int P>
__device__ inline double sum_high(double v) {  // over the second-to-last leg's digit
    if (P == 2) {
        v += dpp_f64<kDppXor2>(v);
    } else {
        v += dpp_f64<kDppRor4>(v);
        v += dpp_f64<kDppRor8>(v);
    }
    return v;
}

__host__ __device__ constexpr bool dpp_shape(int D, int R) {
    return D >= 2 && D <= 4 && R >= 1 && R <= 6 && ipw(D, R - (R < 2 ? R : 2)) <= 16;
}
// tiles per wavefront step: two for small register sets, fewer when the
// tiles' (site, leg) items would exceed one wavefront
__host__ __device__ constexpr int dpp_tiles_in_flight(int D, int R) {
    return ipw(D, R - (R < 2 ? R : 2)) <= 4 ? 2 : 1;  // more register values per lane spill at two
}

template <int D, int R, int KNT>
__device__ __attribute__((noinline)) double ptiles_dpp(const PLayout L, int gl_off, int n_in_group, int chunk,
                                                       int mi, int mo, int scr, int *bad) {
    constexpr int P = D <= 2 ? 2 : 4;
    constexpr int B = P == 2 ? 1 : 2;
    constexpr int T = R < 2 ? R : 2;
    constexpr int NLEG = R - T;
    constexpr int LS = 1 << (B * T);
    constexpr int SPW = 64 / LS;
    constexpr int NL = ipw(D, NLEG);
    constexpr int DT = ipw(D, T);
    constexpr int ND = R * D;
    constexpr int kNT = KNT;  // tiles in flight per wavefront step
    const int lane = threadIdx.x & 63;
    const int slot = lane / LS;
    const int tb = lane - slot * LS;
    const int dlo = tb & (P - 1);                 // digit of leg R-1
    const int dhi = T == 2 ? (tb >> B) : 0;       // digit of leg R-2 (T == 2)
    const bool inseg = dlo < D && dhi < D;
    const int toff = T == 2 ? (dhi % D) * D + dlo % D : dlo % D;
    const int base_pos = chunk * kNT * SPW;
    double tv[kNT][NL];
    double mlo[kNT], mhi[kNT];
    double ml[kNT][NLEG > 0 ? NLEG : 1][D];
    bool act[kNT];
#pragma unroll
    for (int k = 0; k < kNT; ++k) {
        const int pos = base_pos + k * SPW + slot;
        act[k] = inseg && pos < n_in_group;
        const int site = int_at(L.list, gl_off + (pos < n_in_group ? pos : 0));
        const double *tp = tptr_at(L, site);
        const int mb = mi + int_at(L.moff, site);
#pragma unroll
        for (int q = 0; q < NL; ++q) tv[k][q] = dev::gld(tp + q * DT + toff);  // in bounds on every lane
        mlo[k] = p_lds[mb + (R - 1) * D + dlo % D];
        mhi[k] = T == 2 ? p_lds[mb + (R - 2) * D + dhi % D] : 1.0;
#pragma unroll
        for (int j = 0; j < NLEG; ++j)
#pragma unroll
            for (int i = 0; i < D; ++i) ml[k][j][i] = p_lds[mb + j * D + i];
    }
    double *out = p_lds + scr;  // [tile][site][R*D]
#pragma unroll
    for (int k = 0; k < kNT; ++k) {
        const int oslot = (k * SPW + slot) * ND;
        const bool valid = act[k];
        double A = 0.0;
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            double w = 1.0;
#pragma unroll
            for (int j = 0; j < NLEG; ++j) w *= ml[k][j][(q / ipw(D, NLEG - 1 - j)) % D];
            A = fma(tv[k][q], w, A);
        }
        if (!inseg) A = 0.0;  // lanes past the last digit add nothing to the segment sums
        // leg R-1: lanes of one low digit, summed over the high field
        {
            double pm = A * mhi[k];
            if (T == 2) pm = sum_high<P>(pm);
            if (valid && dhi == 0) out[oslot + (R - 1) * D + dlo] = pm;
        }
        // leg R-2: summed over the low field
        if (T == 2) {
            double pm = sum_low<P>(A * mlo[k]);
            if (valid && dlo == 0) out[oslot + (R - 2) * D + dhi] = pm;
        }
        // lead legs: the NLEG*D outputs of a site are per-lane partial sums,
        // reduced jointly over the segment (recursive halving)
        if (NLEG > 0) {
            constexpr int NO = NLEG * D;
            constexpr int NP2 = NO <= 1 ? 1 : (NO <= 2 ? 2 : (NO <= 4 ? 4 : (NO <= 8 ? 8 : 16)));
            const double qt = valid ? mlo[k] * mhi[k] : 0.0;
            // element e = j*D + i: the lane's part of slot j's outgoing entry i
            auto part = [&](int e) {
                if (e >= NO) return 0.0;
                const int j = e / D, i = e % D;
                double sv = 0.0;
#pragma unroll
                for (int q = 0; q < NL; ++q) {
                    if ((q / ipw(D, NLEG - 1 - j)) % D != i) continue;
                    double w = 1.0;
#pragma unroll
                    for (int j2 = 0; j2 < NLEG; ++j2)
                        if (j2 != j) w *= ml[k][j2][(q / ipw(D, NLEG - 1 - j2)) % D];
                    sv = fma(tv[k][q], w, sv);
                }
                return sv * qt;
            };
            double pv[NP2];
            constexpr int M = NP2 > LS ? NP2 / LS : 1;  // totals per lane
            int e;
            bool wr;
            seg_reduce_stream<LS, NP2>(part, pv, tb, e, wr);
            if (wr && base_pos + k * SPW + slot < n_in_group) {
#pragma unroll
                for (int m = 0; m < M; ++m)
                    if (e * M + m < NO) out[oslot + e * M + m] = pv[m];
            }
        }
    }
    wave_sync();
    // Normalisation, element-parallel: item = (tile k, site j in the tile,
    // leg l), its D entries on D of a group of P lanes; the norm, the sign
    // and the residual are group reductions (quad permutations).
    constexpr int NI = kNT * SPW * R;
    constexpr int IPP = 64 / P;  // items per pass
    double res = 0.0;            // this lane's part; the caller reduces over the wave
#pragma unroll
    for (int pass = 0; pass < (NI + IPP - 1) / IPP; ++pass) {
        const int item = pass * IPP + lane / P;
        const int e = lane & (P - 1);
        const int ik = item / (SPW * R);
        const int irem = item - ik * (SPW * R);
        const int ij = irem / R;
        const int il = irem - ij * R;
        const bool live = item < NI && base_pos + ik * SPW + ij < n_in_group;  // uniform over the group
        const bool el = live && e < D;
        double x = 0.0, old = 0.0;
        int idst = 0;
        if (live) {
            const int site = int_at(L.list, gl_off + base_pos + ik * SPW + ij);
            idst = int_at(L.dst, site * kMaxRank + il) + e;
            if (el) {
                x = out[(ik * SPW + ij) * ND + il * D + e];
                old = p_lds[mi + idst];
            }
        }
        double n2 = x * x, sum = x;
        n2 += dpp_f64<kDppXor1>(n2);
        sum += dpp_f64<kDppXor1>(sum);
        if (P == 4) {
            n2 += dpp_f64<kDppXor2>(n2);
            sum += dpp_f64<kDppXor2>(sum);
        }
        const double nrm = sqrt(n2);
        const bool ok = nrm > 0.0 && isfinite(nrm);
        if (live && e == 0 && !ok) *bad = 1;
        const double inv = (sum < 0.0 ? -1.0 : 1.0) / nrm;  // L2 norm, sign fixed so the sum is >= 0
        const double v = x * inv;
        double d1 = el ? fabs(v - old) : 0.0, d2 = el ? fabs(v + old) : 0.0;
        d1 = fmax(d1, dpp_f64<kDppXor1>(d1));
        d2 = fmax(d2, dpp_f64<kDppXor1>(d2));
        if (P == 4) {
            d1 = fmax(d1, dpp_f64<kDppXor2>(d1));
            d2 = fmax(d2, dpp_f64<kDppXor2>(d2));
        }
        if (el && ok) p_lds[mo + idst] = v;
        if (live && ok) res = fmax(res, fmin(d1, d2));
    }
    wave_sync();
    return res;
}

// Messages of the block's network in LDS, addressed by absolute offset.
struct LdsMsg {
    int base;  // LDS index of absolute offset 0
    __device__ double operator()(int o) const { return p_lds[base + o]; }
};

// Register regauge of one tile of a persistent block (kept out of line so
// each shape gets its own register allocation).
template <int D, int R, typename S>
__device__ __attribute__((noinline)) void p_regauge(int cnt, int net, int site_base, int list_off, int first,
                                                    int msg_lds, const SiteRec *__restrict__ sites,
                                                    S *__restrict__ slices, double *__restrict__ site_log,
                                                    int *__restrict__ site_sign, int *status, int scr) {
    const LdsMsg msg{msg_lds};
    auto site_of = [site_base, list_off, first](int j) { return site_base + int_at(list_off, first + j); };
    dev::regauge_reg<D, R, S, dev::rg_passes(D, R)>(cnt, net, site_of, sites, msg, slices, site_log, site_sign,
                                                     status, p_lds + scr);
}

// Regauge on the DPP layout (all legs of dimension D <= 4, same lanes and
// registers as ptiles_dpp).  With a, c the bond's messages, n = a.c and the
// Householder vector u (t = 2/|u|^2) of c, the Appendix-B transform of a slot
// has column 0 equal to g0 (a/n on the bond's first site, c on its second)
// and columns k >= 1 equal to e_k - t u_k u - f_k c, where f = 0 on the first
// site and f_k = (a_k - t u_k (u.a))/n on the second.  Along that slot,
//   T'[0] = W0,  T'[k] = T[k] - t u_k Wu - f_k W0   (k >= 1),
// with W0 = T.g0 and Wu = T.u contracted over the slot: two sums over the
// slot's lane field (DPP all-reduces) or fiber (registers), then an in-lane
// update.  Per (site, slot) one lane builds the record g0[D], u[D], f[D], t
// in the wave's LDS scratch.  NP passes of SPW sites load their tensors
// before any record is built.
template <int D, int R>
__host__ __device__ constexpr int rgd_passes() {
    constexpr int T = R < 2 ? R : 2;
    constexpr int SPW = 64 >> ((D <= 2 ? 1 : 2) * T);
    constexpr int NL = ipw(D, R - T);
    constexpr int a = 16 / NL < 1 ? 1 : (16 / NL > 4 ? 4 : 16 / NL);
    constexpr int b = 512 / (SPW * R * (3 * D + 1));
    return a < b ? a : (b < 1 ? 1 : b);
}
template <int D, int R>
__host__ __device__ constexpr int rgd_sites_per_call() {
    return rgd_passes<D, R>() * (64 >> ((D <= 2 ? 1 : 2) * (R < 2 ? R : 2)));
}

// sites per regauge call of a persistent block for shape (dim, rank)
__host__ __device__ inline int regauge_call_sites(int dim, int rank) {
    switch (dim * 8 + rank) {
#define PNE_SPC(D_, R_) \
    case D_ * 8 + R_: return rgd_sites_per_call<D_, R_>();
        PNE_SPC(2, 1) PNE_SPC(2, 2) PNE_SPC(2, 3) PNE_SPC(2, 4) PNE_SPC(2, 5) PNE_SPC(2, 6) PNE_SPC(3, 1)
        PNE_SPC(3, 2) PNE_SPC(3, 3) PNE_SPC(3, 4) PNE_SPC(4, 1) PNE_SPC(4, 2) PNE_SPC(4, 3) PNE_SPC(4, 4)
#undef PNE_SPC
        default: return dev::regauge_sites_per_call(dim, rank);
    }
}

template <int D, int R, typename S>
__device__ __attribute__((noinline)) void p_regauge_dpp(const PLayout L, int cnt, int net, int site_base, int first,
                                                        int fin, S *__restrict__ slices,
                                                        double *__restrict__ site_log, int *__restrict__ site_sign,
                                                        int *status, int scr) {
    constexpr int P = D <= 2 ? 2 : 4;
    constexpr int B = P == 2 ? 1 : 2;
    constexpr int T = R < 2 ? R : 2;
    constexpr int NLEG = R - T;
    constexpr int LS = 1 << (B * T);
    constexpr int SPW = 64 / LS;
    constexpr int NL = ipw(D, NLEG);
    constexpr int DT = ipw(D, T);
    constexpr int GR = 3 * D + 1;
    constexpr int NP = rgd_passes<D, R>();
    const int lane = threadIdx.x & 63;
    const int slot = lane / LS;
    const int tb = lane - slot * LS;
    const int dlo = tb & (P - 1);
    const int dhi = T == 2 ? (tb >> B) : 0;
    const bool inseg = dlo < D && dhi < D;
    const int toff = T == 2 ? (dhi % D) * D + dlo % D : dlo % D;
    // every pass's tensor values first: the call's only global loads
    double v[NP][NL];
    int ls[NP];
    bool act[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int j = k * SPW + slot;
        act[k] = inseg && j < cnt;
        ls[k] = int_at(L.list, first + (j < cnt ? j : 0));
        const double *tp = tptr_at(L, ls[k]);
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const double x = dev::gld(tp + q * DT + toff);  // in bounds on every lane
            v[k][q] = act[k] ? x : 0.0;
        }
    }
    double *G = p_lds + scr;  // [site][slot][GR]
    wave_sync();              // the wave's previous call has finished reading G
    for (int j = lane; j < cnt * R; j += 64) {
        const int s = j / R;
        const int l = j - s * R;
        const int loc = int_at(L.list, first + s);
        const bool vs = (int_at(L.vside, loc) >> l) & 1;
        const int pin = fin + int_at(L.moff, loc) + l * D;
        const int pout = fin + int_at(L.dst, loc * kMaxRank + l);
        double a[D], c[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double x = p_lds[pin + i], y = p_lds[pout + i];
            a[i] = vs ? y : x;
            c[i] = vs ? x : y;
        }
        const dev::LegGauge g = dev::leg_gauge_setup(a, c, D);
        double *rec = G + j * GR;
        if (!g.ok) {
            atomicMin(status, -4);
#pragma unroll
            for (int i = 0; i < D; ++i) {
                rec[i] = i == 0 ? 1.0 : 0.0;
                rec[D + i] = 0.0;
                rec[2 * D + i] = 0.0;
            }
            rec[3 * D] = 0.0;
            continue;
        }
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double ui = i == 0 ? g.u0 : c[i] * g.inv_nc;
            rec[i] = vs ? c[i] : a[i] * g.inv_n;
            rec[D + i] = ui;
            rec[2 * D + i] = (vs && i > 0) ? (a[i] - g.t * ui * g.ua) * g.inv_n : 0.0;
        }
        rec[3 * D] = g.t;
    }
    wave_sync();
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        if (k * SPW >= cnt) break;
        const int j = k * SPW + slot;
        const double *Gs = G + (j < cnt ? j : 0) * R * GR;
        // register (lead) legs: contractions along each fiber
#pragma unroll
        for (int jl = 0; jl < NLEG; ++jl) {
            const double *g = Gs + jl * GR;
            const double t = g[3 * D];
            constexpr int dummy = 0;
            (void)dummy;
#pragma unroll
            for (int q0 = 0; q0 < NL; ++q0) {
                const int stride = ipw(D, NLEG - 1 - jl);
                if ((q0 / stride) % D != 0) continue;
                double w0 = 0.0, wu = 0.0;
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    w0 = fma(v[k][q0 + i * stride], g[i], w0);
                    wu = fma(v[k][q0 + i * stride], g[D + i], wu);
                }
                v[k][q0] = w0;
#pragma unroll
                for (int kk = 1; kk < D; ++kk)
                    v[k][q0 + kk * stride] = v[k][q0 + kk * stride] - t * g[D + kk] * wu - g[2 * D + kk] * w0;
            }
        }
        // lane legs (leg R-1 on the low field, leg R-2 on the high field),
        // one register value at a time, each stored as soon as it is final;
        // value 0 carries the vacuum factor T'[0,...,0] in the segment's
        // first lane
        double g0m[T], gum[T], cum[T], cfm[T];
        bool zero_digit[T];
#pragma unroll
        for (int m = 0; m < T; ++m) {
            const double *g = Gs + (R - 1 - m) * GR;
            const int d = m == 0 ? dlo : dhi;
            const bool dv = d < D;
            const int dd = dv ? d : 0;
            g0m[m] = dv ? g[dd] : 0.0;
            gum[m] = dv ? g[D + dd] : 0.0;
            cum[m] = dv ? g[3 * D] * g[D + dd] : 0.0;
            cfm[m] = dv ? g[2 * D + dd] : 0.0;
            zero_digit[m] = d == 0;
        }
        const int64_t so = reinterpret_cast<const int64_t *>(p_lds + L.soff)[ls[k]];
        double z = 0.0, iz = 0.0;
        bool ok = false;
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            double x = v[k][q];
#pragma unroll
            for (int m = 0; m < T; ++m) {
                double w0 = x * g0m[m], wu = x * gum[m];
                if (m == 0) {
                    w0 = sum_low<P>(w0);
                    wu = sum_low<P>(wu);
                } else {
                    w0 = sum_high<P>(w0);
                    wu = sum_high<P>(wu);
                }
                x = zero_digit[m] ? w0 : x - cum[m] * wu - cfm[m] * w0;
            }
            if (q == 0) {
                z = __shfl(x, slot * LS, 64);
                ok = (fabs(z) > 0.0) && isfinite(z);
                iz = ok ? 1.0 / z : 0.0;
            }
            if (act[k]) dev::SliceIO<S>::store(slices, so + q * DT + toff, x * iz);
        }
        if (tb == 0 && j < cnt) {
            dev::gst(site_log + site_base + ls[k], ok ? log(fabs(z)) : 0.0);
            dev::gst(site_sign + site_base + ls[k], z < 0.0 ? -1 : 1);
            if (!ok) atomicMin(status, -4);
        }
    }
}

// The scalar and cycle clusters of one network, one instance per thread of
// the block (kept out of line: its registers stay apart from the BP loop's).
template <typename S, int NT>
__device__ __attribute__((noinline)) void p_clusters(int class_begin, int n_classes, int64_t w_base,
                                                     int64_t slice_base, const ClassDesc *__restrict__ classes,
                                                     const S *__restrict__ slices, double *__restrict__ w) {
    for (int c = class_begin; c < class_begin + n_classes; ++c) {
        const ClassDesc cd = classes[c];
        const int per = cd.loop_e ? cd.n_verts : cd.n_steps;
        for (int k = threadIdx.x; k < cd.n_inst; k += NT) {
            const InstStep *rec = cd.tab + (int64_t)k * per;
            dev::gst(w + w_base + dev::gld(cd.iw + k), (double)dev::fast_term<S>(cd, rec, slices, slice_base));
        }
    }
}

// NT threads per block: kPThreads for most networks, kPSmallThreads for
// networks of at most a batch-chosen number of sites (more of them share a
// CU).  WPE: the fewest waves per SIMD the register allocation must allow;
// 4 caps a lane at 128 VGPRs (two 512-thread blocks per CU), 2 at 256 (one
// block per CU, no spills, twice the LDS per block).
// A double that every lane of the wave holds, read from the first lane, so
// that the compiler can keep it (and what is derived from it) in SGPRs.
__device__ __forceinline__ double uniform_double(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

template <typename S, int NT, int WPE>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_bp_persistent(const FusedNet *__restrict__ fnets, const FusedGroup *__restrict__ groups,
                const int *__restrict__ site_list, const SiteRec *__restrict__ sites, double *msg0, NetState *st,
                double tol, int max_iter, int stall, double floor_tol, S *__restrict__ slices,
                double *__restrict__ site_log,
                int *__restrict__ site_sign, int rg_enabled, const ClassDesc *__restrict__ classes,
                double *__restrict__ w,
                const CombineRec *__restrict__ crecs, const GeoRec *__restrict__ geos,
                const Bucket *__restrict__ buckets, const int *__restrict__ pair_a, const int *__restrict__ pair_b,
                const PairCat *__restrict__ cats, NetResult *__restrict__ results) {
    constexpr int NW = NT / 64;
    const FusedNet fn = fnets[blockIdx.x];
    if (fn.prio) __builtin_amdgcn_s_setprio(2);
    NetState *ns = st + fn.net;
    const unsigned long long t_start = wall_clock64();
    __shared__ double s_res[2 * NW];
    // a singular message in step k sets s_bad[k & 1]: every wave reads the
    // slot of its own step after that step's barrier, so all waves leave the
    // loop at the same step (a fast wave's next step writes the other slot)
    __shared__ int s_bad[2];
    __shared__ int s_status;  // the network's status this run (lowered with LDS atomics)
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int ns_ = fn.n_sites;
    const bool rb = fn.colors == 2;  // red-black schedule: one buffer, updated in place
    PLayout L;
    L.b0 = 0;
    L.b1 = rb ? 0 : fn.msg_size;
    L.tptr = (rb ? 1 : 2) * fn.msg_size;
    L.moff = L.tptr + ns_;
    L.dst = L.moff + (ns_ + 1) / 2;
    L.list = L.dst + (ns_ * kMaxRank + 1) / 2;
    L.vside = L.list + (ns_ + 1) / 2;
    L.soff = L.vside + (ns_ + 1) / 2;
    L.scr = L.soff + ns_;
    const int scr = L.scr + wave * fn.scratch;
    // uniform initial messages 1/sqrt(d): each site fills its incoming slots
    for (int s = tid; s < ns_; s += NT) {
        const SiteRec &r = sites[fn.site_base + s];
        for (int l = 0; l < r.rank; ++l) {
            const double v = 1.0 / sqrt((double)r.dim[l]);
            double *m = p_lds + (r.msg_off - fn.msg_base) + r.moff[l];
            for (int k = 0; k < r.dim[l]; ++k) m[k] = v;
        }
        reinterpret_cast<const double **>(p_lds + L.tptr)[s] = r.t;
        reinterpret_cast<int *>(p_lds + L.moff)[s] = r.msg_off - fn.msg_base;
        for (int l = 0; l < kMaxRank; ++l)
            reinterpret_cast<int *>(p_lds + L.dst)[s * kMaxRank + l] = l < r.rank ? r.dst[l] - fn.msg_base : 0;
        reinterpret_cast<int *>(p_lds + L.list)[s] = site_list[fn.list_begin + s];
        reinterpret_cast<int *>(p_lds + L.vside)[s] = r.vside_mask;
        reinterpret_cast<int64_t *>(p_lds + L.soff)[s] = r.slice_off;
    }
    if (tid == 0) {
        s_bad[0] = 0;
        s_bad[1] = 0;
        s_status = 0;
    }
    __syncthreads();
    int sweep = 0;
    double r = 0.0, r_prev = 0.0;
    // smallest residual so far (red-black: of the last two steps) and the
    // step that reached it, for the rounding-floor stop
    double r_best = INFINITY;
    int best_at = -1;
    bool conv = false;
    for (sweep = 0; sweep < max_iter; ++sweep) {
        // Jacobi: read buffer sweep&1, write the other.  Red-black: sites of
        // colour sweep&1 read their incoming messages and overwrite their
        // outgoing ones (the incoming messages of the other colour), so no
        // message is read and written in the same step.
        const int mi = (sweep & 1) ? L.b1 : L.b0;
        const int mo = (sweep & 1) ? L.b0 : L.b1;
        double wres = 0.0;
        int *bad_slot = &s_bad[sweep & 1];
        // chunks of all groups in one sequence, dealt round-robin to the waves
        int cbase = 0;
        for (int g = 0; g < fn.n_groups; ++g) {
            const FusedGroup gr = groups[fn.group_begin + g];
            if (rb && gr.color != (sweep & 1)) continue;
            const int per_chunk = gr.nt * gr.spw;
            const int nchunks = (gr.n_sites + per_chunk - 1) / per_chunk;
            const int c0 = ((wave - cbase) % NW + NW) % NW;
            cbase += nchunks;
            for (int c = c0; c < nchunks; c += NW) {
                double tr = 0.0;
                // DPP shapes: one or two tiles in flight (chosen per batch); the
                // other shapes have one fixed tiling
#define PNE_PT2(D_, R_)                                                                   \
    case (D_ * 8 + R_) * 4 + 1:                                                           \
        tr = ptiles_dpp<D_, R_, 1>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, bad_slot); \
        break;                                                                            \
    case (D_ * 8 + R_) * 4 + 2:                                                           \
        tr = ptiles_dpp<D_, R_, 2>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, bad_slot); \
        break;
#define PNE_PT1(D_, R_)                                                             \
    case (D_ * 8 + R_) * 4 + tiles_in_flight(ipw(D_, R_ - ((6 / (D_ <= 2 ? 1 : (D_ <= 4 ? 2 : 3))) < R_ ? (6 / (D_ <= 2 ? 1 : (D_ <= 4 ? 2 : 3))) : R_))): \
        tr = ptiles<D_, R_>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, bad_slot);  \
        break;
                switch ((gr.dc * 8 + gr.rank) * 4 + gr.nt) {
                    PNE_PT2(2, 1) PNE_PT2(2, 2) PNE_PT2(2, 3) PNE_PT2(2, 4) PNE_PT2(2, 5) PNE_PT2(2, 6)
                    PNE_PT2(3, 1) PNE_PT2(3, 2) PNE_PT2(3, 3) PNE_PT2(3, 4)
                    PNE_PT2(4, 1) PNE_PT2(4, 2) PNE_PT2(4, 3) PNE_PT2(4, 4)
                    PNE_PT1(3, 5) PNE_PT1(4, 5) PNE_PT1(5, 1) PNE_PT1(5, 2) PNE_PT1(5, 3)
                    PNE_PT1(6, 1) PNE_PT1(6, 2) PNE_PT1(6, 3)
                    default: break;
                }
#undef PNE_PT1
#undef PNE_PT2
                wres = fmax(wres, tr);
            }
        }
        // the tiles return per-lane parts; one wave reduction per step.  The
        // two residual slots alternate, so a slot is rewritten only after a
        // later barrier that every wave reaches after reading it.
        wres = wave_max_p(wres);
        double *slot = s_res + (sweep & 1) * NW;
        if ((tid & 63) == 0) slot[wave] = wres;
        __syncthreads();
        r = slot[0];
        for (int w = 1; w < NW; ++w) r = fmax(r, slot[w]);
        // both slots are still clear whenever the loop goes on
        if (*bad_slot) break;
        // red-black: both colours' latest updates must be within tol
        if (r <= tol && (!rb || (sweep > 0 && r_prev <= tol))) {
            conv = true;
            break;
        }
        // the same value in every lane: keep the record in scalar registers
        const double rr = uniform_double(rb ? fmax(r, r_prev) : r);
        if (rr < r_best) {
            r_best = rr;
            best_at = sweep;
        } else if (stall > 0 && r_best <= floor_tol && sweep - best_at >= stall) {
            conv = true;
            break;
        }
        r_prev = r;
    }
    const int last = sweep < max_iter ? sweep : max_iter - 1;
    const int fin = rb ? L.b0 : ((last & 1) ? L.b0 : L.b1);
    for (int e = tid; e < fn.msg_size; e += NT) msg0[fn.msg_base + e] = p_lds[fin + e];
    if (tid == 0) {
        ns->stop = last;
        ns->iters = last + 1;
        ns->parity = 0;
        ns->residual = rb ? fmax(r, r_prev) : r;
        ns->converged = conv ? 1 : 0;
        if (s_bad[0] | s_bad[1]) s_status = -4;
        ns->status = s_status;
        ns->t_start = t_start;
        ns->t_bp = wall_clock64();
        ns->t_rg = ns->t_bp;
    }
    if (!fn.rg_inline || !rg_enabled) return;
    // Gauge and slices (Appendix B; Sec. VI) straight from the final
    // messages in LDS: register-path tiles of each shape group dealt to the
    // waves, each wave's transform table in its BP scratch (free after the
    // last sweep's barrier).
    const int msg_lds = fin - fn.msg_base;
    int tbase = 0;
    for (int g = 0; g < fn.n_groups; ++g) {
        const FusedGroup gr = groups[fn.group_begin + g];
        const int spt = regauge_call_sites(gr.dc, gr.rank);
        const int ntl = (gr.n_sites + spt - 1) / spt;
        const int t0 = ((wave - tbase) % NW + NW) % NW;
        tbase += ntl;
        for (int t = t0; t < ntl; t += NW) {
            const int first = gr.list_off + t * spt;
            const int cnt = min(spt, gr.n_sites - t * spt);
#define PNE_PRG(D_, R_)                                                                                    \
    case D_ * 8 + R_:                                                                                     \
        p_regauge<D_, R_, S>(cnt, fn.net, fn.site_base, L.list, first, msg_lds, sites, slices, site_log, \
                             site_sign, &s_status, scr);                                                         \
        break;
#define PNE_PRGD(D_, R_)                                                                                    \
    case D_ * 8 + R_:                                                                                      \
        p_regauge_dpp<D_, R_, S>(L, cnt, fn.net, fn.site_base, first, fin, slices, site_log, site_sign,      \
                                 &s_status, scr);                                                                     \
        break;
            switch (gr.dc * 8 + gr.rank) {
                PNE_PRGD(2, 1) PNE_PRGD(2, 2) PNE_PRGD(2, 3) PNE_PRGD(2, 4) PNE_PRGD(2, 5) PNE_PRGD(2, 6)
                PNE_PRGD(3, 1) PNE_PRGD(3, 2) PNE_PRGD(3, 3) PNE_PRGD(3, 4) PNE_PRGD(4, 1) PNE_PRGD(4, 2)
                PNE_PRGD(4, 3) PNE_PRGD(4, 4)
                PNE_PRG(5, 1) PNE_PRG(5, 2) PNE_PRG(6, 1) PNE_PRG(6, 2)
                default: break;
            }
#undef PNE_PRG
#undef PNE_PRGD
        }
    }
    __syncthreads();  // the network's slices and vacuum factors are written
    if (tid == 0) {
        ns->t_rg = wall_clock64();
        ns->status = s_status;  // lowered by the gauge on a singular bond or vacuum factor
    }
    if (!fn.cl_fused) return;
    // Clusters of the network (scalar and cycle classes: one instance per
    // thread, slices just written by this block) and its FP64 term sum.
    p_clusters<S, NT>(fn.class_begin, fn.n_classes, fn.w_base, reinterpret_cast<const int64_t *>(p_lds + L.soff)[0],
                  classes, slices, w);
    __syncthreads();
    const CombineRec cr = crecs[fn.net];
    dev::combine_closed<NT, S>(fn.net, cr, geos[cr.geo], buckets, pair_a, pair_b, cats, w, site_log, site_sign,
                               sites, slices, s_status, results, p_lds + L.scr);
}

}  // namespace

// doubles of dynamic LDS for a persistent block (see PLayout)
size_t bp_persistent_lds_doubles(int msg_size, int n_sites, int scratch_per_wave, int n_buffers, bool small) {
    const int waves = small ? kPSmallThreads / 64 : kPWaves;
    return (size_t)n_buffers * msg_size + (size_t)n_sites + (size_t)(n_sites + 1) / 2 +
           (size_t)(n_sites * kMaxRank + 1) / 2 + 2 * (size_t)((n_sites + 1) / 2) + (size_t)n_sites +
           (size_t)waves * scratch_per_wave;
}

// Shapes whose gauge and slices the persistent block builds itself: the DPP
// layout (D <= 4, up to 16 register values) or the shuffle register path.
bool bp_persistent_regauge_supported(int dim, int rank) {
    return dpp_shape(dim, rank) || regauge_reg_supported(dim, rank);
}

int bp_persistent_regauge_table(int dim, int rank) {
    if (dpp_shape(dim, rank)) return regauge_call_sites(dim, rank) * rank * (3 * dim + 1);
    return dev::regauge_call_table(dim, rank);
}

int bp_persistent_tiles_in_flight(int dim, int rank) {
    if (dpp_shape(dim, rank)) return dpp_tiles_in_flight(dim, rank);
    const int B = dim <= 2 ? 1 : (dim <= 4 ? 2 : 3);
    const int T = (6 / B) < rank ? (6 / B) : rank;
    return tiles_in_flight(ipw(dim, rank - T));
}

int bp_persistent_sites_per_tile(int dim, int rank) {
    if (dpp_shape(dim, rank)) {
        const int B = dim <= 2 ? 1 : 2;
        const int T = rank < 2 ? rank : 2;
        return 64 >> (B * T);
    }
    return bp_reg_sites_per_tile(dim, rank);
}

bool bp_persistent_tiles_tunable(int dim, int rank) { return dpp_shape(dim, rank); }

int bp_persistent_scratch(int spw, int rank, int dim, int nt) {
    return nt * spw * rank * dim;
}

template <int NT, int WPE>
void launch_fused_w(const DeviceBatch &b, const FusedNet *fused, int n, size_t lds, double tol, int max_iter,
                    hipStream_t s) {
    switch (b.precision) {
        case 0:
            hipLaunchKernelGGL((k_bp_persistent<double, NT, WPE>), dim3(n), dim3(NT), lds, s, fused, b.fgroups,
                               b.fsite_list, b.sites, b.msg0, b.state, tol, max_iter, b.bp_stall, b.bp_floor, (double *)b.slices,
                               b.site_log, b.site_sign, b.fused_regauge, b.classes, b.w, b.crec, b.geos,
                               b.buckets, b.pair_a, b.pair_b, b.pair_cats, b.results);
            break;
        case 1:
            hipLaunchKernelGGL((k_bp_persistent<float, NT, WPE>), dim3(n), dim3(NT), lds, s, fused, b.fgroups,
                               b.fsite_list, b.sites, b.msg0, b.state, tol, max_iter, b.bp_stall, b.bp_floor, (float *)b.slices,
                               b.site_log, b.site_sign, b.fused_regauge, b.classes, b.w, b.crec, b.geos,
                               b.buckets, b.pair_a, b.pair_b, b.pair_cats, b.results);
            break;
        default:
            hipLaunchKernelGGL((k_bp_persistent<uint16_t, NT, WPE>), dim3(n), dim3(NT), lds, s, fused, b.fgroups,
                               b.fsite_list, b.sites, b.msg0, b.state, tol, max_iter, b.bp_stall, b.bp_floor, (uint16_t *)b.slices,
                               b.site_log, b.site_sign, b.fused_regauge, b.classes, b.w, b.crec, b.geos,
                               b.buckets, b.pair_a, b.pair_b, b.pair_cats, b.results);
            break;
    }
}

template <int NT>
void launch_fused_nt(const DeviceBatch &b, const FusedNet *fused, int n, size_t lds, double tol, int max_iter,
                     hipStream_t s) {
    if (b.reg_budget)
        launch_fused_w<NT, 2>(b, fused, n, lds, tol, max_iter, s);
    else
        launch_fused_w<NT, 4>(b, fused, n, lds, tol, max_iter, s);
}

hipError_t launch_fused(const DeviceBatch &b, double tol, int max_iter, hipStream_t s) {
    const int n_large = b.n_fused - b.n_fused_small - b.n_fused_big;
    if (n_large > 0) launch_fused_nt<kPThreads>(b, b.fused, n_large, b.fused_lds, tol, max_iter, s);
    if (b.n_fused_small > 0)
        launch_fused_nt<kPSmallThreads>(b, b.fused + n_large, b.n_fused_small, b.fused_lds_small, tol, max_iter, s);
    // networks whose LDS only the one-block-per-CU kernel has
    if (b.n_fused_big > 0)
        launch_fused_w<kPThreads, 2>(b, b.fused + n_large + b.n_fused_small, b.n_fused_big, b.fused_lds_big, tol,
                                     max_iter, s);
    return hipGetLastError();
}

}  // namespace pne
