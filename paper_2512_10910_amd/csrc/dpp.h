// Cross-lane sums of doubles on gfx950 by data-parallel-primitive (DPP)
// moves: a lane reads a partner inside its 16-lane row through the VALU, with
// no LDS permute.  Only sums of values every lane holds; the result is the
// same in every lane of the group because each butterfly stage adds two
// partial sums in either order.
#pragma once

#include <hip/hip_runtime.h>

namespace pne {
namespace dpp {

// A lane's partner lane ^ MASK within its 16-lane row, for MASK 15, 7, 3, 1
// (row_mirror, row_half_mirror, quad_perm [3,2,1,0], quad_perm [1,0,3,2]):
// full permutations of a row, so no lane reads outside it.
template <int MASK>
__device__ inline double row_partner(double v) {
    static_assert(MASK == 15 || MASK == 7 || MASK == 3 || MASK == 1, "row partner mask");
    constexpr int ctrl = MASK == 15 ? 0x140 : (MASK == 7 ? 0x141 : (MASK == 3 ? 0x1B : 0xB1));
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// The lane (lane + N) mod 16 of the lane's row (row_ror:N; N = 4 or 8).
template <int N>
__device__ inline double row_ror(double v) {
    static_assert(N == 4 || N == 8, "row rotation");
    constexpr int ctrl = 0x120 + N;
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sum over the lanes that differ from this one only in lane bits
// [LO, LO + NB): DPP moves where the bits lie inside a row, cross-row
// shuffles for bits 4 and 5.
template <int LO, int NB>
__device__ inline double bits_sum(double v) {
    if constexpr (LO == 0 && NB == 1) {
        v += row_partner<1>(v);
    } else if constexpr (LO == 0 && NB == 2) {
        v += row_partner<3>(v);
        v += row_partner<1>(v);
    } else if constexpr (LO == 0 && NB == 3) {
        v += row_partner<7>(v);
        v += row_partner<3>(v);
        v += row_partner<1>(v);
    } else if constexpr (LO == 2 && NB == 2) {  // lanes i, i + 4, i + 8, i + 12 of the row
        v += row_ror<4>(v);
        v += row_ror<8>(v);
    } else if constexpr (LO == 3 && NB == 3) {
        v += row_ror<8>(v);
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
    } else {
#pragma unroll
        for (int b = LO; b < LO + NB; ++b) v += __shfl_xor(v, 1 << b, 64);
    }
    return v;
}

// Sum over the lane's 16-lane row: a butterfly over the four lane bits.
__device__ inline double row_sum(double v) {
    v += row_partner<15>(v);
    v += row_partner<7>(v);
    v += row_partner<3>(v);
    v += row_partner<1>(v);
    return v;
}

// Pair stage of a recursive halving over one lane bit: the lane keeps value
// `lo` or `hi` as its bit is 0 or 1 and adds the partner's copy of it; the
// partner (opposite bit, same index set) receives the other one.
template <int MASK>
__device__ inline double halve(double lo, double hi, bool bit) {
    const double keep = bit ? hi : lo;
    return keep + row_partner<MASK>(bit ? lo : hi);
}

// Joint sums of N <= 16 values per lane over the wavefront by recursive
// halving inside each row (lane bits 3, 2, 1, 0 with the partners lane ^ 15,
// ^ 7, ^ 3, ^ 1, each of which keeps the higher bits), then across the four
// rows.  Lane l ends with the wavefront's sum of value l & 15 (0 where
// l & 15 >= N): 15 DPP moves and two shuffles in place of N wave_sum calls.
template <int N>
__device__ inline double wave_sums16(const double (&v)[N], int lane) {
    static_assert(N >= 1 && N <= 16, "at most 16 values");
    double a[8], b[4], c[2];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = j < N ? halve<15>(v[j], j + 8 < N ? v[j + 8] : 0.0, lane & 8) : 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = j < N ? halve<7>(a[j], a[j + 4], lane & 4) : 0.0;
#pragma unroll
    for (int j = 0; j < 2; ++j) c[j] = j < N ? halve<3>(b[j], b[j + 2], lane & 2) : 0.0;
    double d = halve<1>(c[0], c[1], lane & 1);
    d += __shfl_xor(d, 16, 64);
    d += __shfl_xor(d, 32, 64);
    return d;
}

// Sum over the wavefront: the row butterfly, then across the four rows.
__device__ inline double wave_sum(double v) {
    v = row_sum(v);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

}  // namespace dpp
}  // namespace pne
