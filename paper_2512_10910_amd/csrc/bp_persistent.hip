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

namespace pne {

namespace {

constexpr int kPThreads = 512;
constexpr int kPWaves = kPThreads / 64;
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
        for (int q = 0; q < NL; ++q) tv[k][q] = act[k] ? tp[q * DT + toff] : 0.0;
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
        const double sg = sum < 0.0 ? -1.0 : 1.0;
        double d1 = 0.0, d2 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double v = sg * (raw[i] / nrm);
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
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
constexpr int kDppXor1 = 0xB1;    // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;    // quad_perm [2,3,0,1]
constexpr int kDppRor4 = 0x124;   // row_ror:4
constexpr int kDppRor8 = 0x128;   // row_ror:8

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
    return (tiles_in_flight(ipw(D, R - (R < 2 ? R : 2))) == 2 &&
            2 * (64 >> ((D <= 2 ? 1 : 2) * (R < 2 ? R : 2))) * R <= 64)
               ? 2
               : 1;
}

template <int D, int R>
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
    constexpr int kNT = dpp_tiles_in_flight(D, R);
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
        for (int q = 0; q < NL; ++q) tv[k][q] = act[k] ? tp[q * DT + toff] : 0.0;
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
        // lead legs: summed over the whole segment
        if (NLEG > 0) {
            const double qt = valid ? mlo[k] * mhi[k] : 0.0;
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
                    sv = sum_low<P>(sv * qt);
                    if (T == 2) sv = sum_high<P>(sv);
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
        const double sg = sum < 0.0 ? -1.0 : 1.0;
        double d1 = 0.0, d2 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const double v = sg * (raw[i] / nrm);
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

__global__ void __launch_bounds__(kPThreads) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_bp_persistent(const FusedNet *__restrict__ fnets, const FusedGroup *__restrict__ groups,
                const int *__restrict__ site_list, const SiteRec *__restrict__ sites, double *msg0, NetState *st,
                double tol, int max_iter) {
    const FusedNet fn = fnets[blockIdx.x];
    NetState *ns = st + fn.net;
    __shared__ double s_res[kPWaves];
    __shared__ int s_bad;
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
    L.scr = L.list + (ns_ + 1) / 2;
    const int scr = L.scr + wave * fn.scratch;
    for (int e = tid; e < fn.msg_size; e += kPThreads) p_lds[e] = msg0[fn.msg_base + e];
    for (int s = tid; s < ns_; s += kPThreads) {
        const SiteRec &r = sites[fn.site_base + s];
        reinterpret_cast<const double **>(p_lds + L.tptr)[s] = r.t;
        reinterpret_cast<int *>(p_lds + L.moff)[s] = r.msg_off - fn.msg_base;
        for (int l = 0; l < kMaxRank; ++l)
            reinterpret_cast<int *>(p_lds + L.dst)[s * kMaxRank + l] = l < r.rank ? r.dst[l] - fn.msg_base : 0;
        reinterpret_cast<int *>(p_lds + L.list)[s] = site_list[fn.list_begin + s];
    }
    if (tid == 0) s_bad = 0;
    __syncthreads();
    int sweep = 0;
    double r = 0.0, r_prev = 0.0;
    bool conv = false;
    for (sweep = 0; sweep < max_iter; ++sweep) {
        // Jacobi: read buffer sweep&1, write the other.  Red-black: sites of
        // colour sweep&1 read their incoming messages and overwrite their
        // outgoing ones (the incoming messages of the other colour), so no
        // message is read and written in the same step.
        const int mi = (sweep & 1) ? L.b1 : L.b0;
        const int mo = (sweep & 1) ? L.b0 : L.b1;
        double wres = 0.0;
        // chunks of all groups in one sequence, dealt round-robin to the waves
        int cbase = 0;
        for (int g = 0; g < fn.n_groups; ++g) {
            const FusedGroup gr = groups[fn.group_begin + g];
            if (rb && gr.color != (sweep & 1)) continue;
            const int per_chunk = gr.nt * gr.spw;
            const int nchunks = (gr.n_sites + per_chunk - 1) / per_chunk;
            const int c0 = ((wave - cbase) % kPWaves + kPWaves) % kPWaves;
            cbase += nchunks;
            for (int c = c0; c < nchunks; c += kPWaves) {
                double tr = 0.0;
                switch (gr.dc * 8 + gr.rank) {
                    case 17: tr = ptiles_dpp<2, 1>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 18: tr = ptiles_dpp<2, 2>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 19: tr = ptiles_dpp<2, 3>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 20: tr = ptiles_dpp<2, 4>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 21: tr = ptiles_dpp<2, 5>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 22: tr = ptiles_dpp<2, 6>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 25: tr = ptiles_dpp<3, 1>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 26: tr = ptiles_dpp<3, 2>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 27: tr = ptiles_dpp<3, 3>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 28: tr = ptiles_dpp<3, 4>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 29: tr = ptiles<3, 5>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 33: tr = ptiles_dpp<4, 1>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 34: tr = ptiles_dpp<4, 2>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 35: tr = ptiles_dpp<4, 3>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 36: tr = ptiles_dpp<4, 4>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 37: tr = ptiles<4, 5>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 41: tr = ptiles<5, 1>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 42: tr = ptiles<5, 2>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 43: tr = ptiles<5, 3>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 49: tr = ptiles<6, 1>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 50: tr = ptiles<6, 2>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    case 51: tr = ptiles<6, 3>(L, gr.list_off, gr.n_sites, c, mi, mo, scr, &s_bad); break;
                    default: break;
                }
                wres = fmax(wres, tr);
            }
        }
        if ((tid & 63) == 0) s_res[wave] = wres;
        __syncthreads();
        r = s_res[0];
        for (int w = 1; w < kPWaves; ++w) r = fmax(r, s_res[w]);
        const int bad = s_bad;
        __syncthreads();
        if (bad) break;
        // red-black: both colours' latest updates must be within tol
        if (r <= tol && (!rb || (sweep > 0 && r_prev <= tol))) {
            conv = true;
            break;
        }
        r_prev = r;
    }
    const int last = sweep < max_iter ? sweep : max_iter - 1;
    const int fin = rb ? L.b0 : ((last & 1) ? L.b0 : L.b1);
    for (int e = tid; e < fn.msg_size; e += kPThreads) msg0[fn.msg_base + e] = p_lds[fin + e];
    if (tid == 0) {
        ns->stop = last;
        ns->iters = last + 1;
        ns->parity = 0;
        ns->residual = rb ? fmax(r, r_prev) : r;
        ns->converged = conv ? 1 : 0;
        if (s_bad) ns->status = -4;
    }
}

}  // namespace

// doubles of dynamic LDS for a persistent block (see PLayout)
size_t bp_persistent_lds_doubles(int msg_size, int n_sites, int scratch_per_wave, int n_buffers) {
    return (size_t)n_buffers * msg_size + (size_t)n_sites + (size_t)(n_sites + 1) / 2 +
           (size_t)(n_sites * kMaxRank + 1) / 2 + (size_t)(n_sites + 1) / 2 + (size_t)kPWaves * scratch_per_wave;
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

int bp_persistent_scratch(int spw, int rank, int dim) {
    return bp_persistent_tiles_in_flight(dim, rank) * spw * rank * dim;
}

hipError_t launch_fused(const DeviceBatch &b, double tol, int max_iter, hipStream_t s) {
    if (!b.n_fused) return hipSuccess;
    hipLaunchKernelGGL(k_bp_persistent, dim3(b.n_fused), dim3(kPThreads), b.fused_lds, s, b.fused, b.fgroups,
                       b.fsite_list, b.sites, b.msg0, b.state, tol, max_iter);
    return hipGetLastError();
}

}  // namespace pne
