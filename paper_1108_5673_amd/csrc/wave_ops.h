// wave_ops.h -- wavefront-level helpers for 64-lane CDNA wavefronts.
#pragma once

#include <hip/hip_runtime.h>

namespace pwa {

__device__ inline int lane_id() { return threadIdx.x & 63; }

// Broadcast lane `src` (wave-uniform) of a double to every lane, through
// scalar registers.
__device__ inline double readlane_f64(double x, int src)
{
    int lo = __double2loint(x);
    int hi = __double2hiint(x);
    lo = __builtin_amdgcn_readlane(lo, src);
    hi = __builtin_amdgcn_readlane(hi, src);
    return __hiloint2double(hi, lo);
}

// Sum over all 64 lanes with a fixed xor butterfly: every lane ends with the
// same, run-to-run reproducible value.
__device__ inline double wave_allsum(double x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
    return x;
}

__device__ inline int wave_allsum_int(int x)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
    return x;
}

// ---- cross-lane exchanges of doubles --------------------------------------
// gfx950 permlane swaps exchange whole lane halves between two registers:
//   swap32(a, b): lanes 32..63 of a  <->  lanes 0..31 of b
//   swap16(a, b): lanes 16..31 of a  <->  lanes 0..15 of b, and 48..63 <-> 32..47
// so that afterwards a + b holds, in the lower half of each pair of lane
// groups, the pairwise sum of a and, in the upper half, that of b.
__device__ inline void swap32_f64(double& a, double& b)
{
    auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a),
                                               (unsigned)__double2loint(b), false, false);
    auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a),
                                               (unsigned)__double2hiint(b), false, false);
    a = __hiloint2double((int)hi[0], (int)lo[0]);
    b = __hiloint2double((int)hi[1], (int)lo[1]);
}

__device__ inline void swap16_f64(double& a, double& b)
{
    auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a),
                                               (unsigned)__double2loint(b), false, false);
    auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a),
                                               (unsigned)__double2hiint(b), false, false);
    a = __hiloint2double((int)hi[0], (int)lo[0]);
    b = __hiloint2double((int)hi[1], (int)lo[1]);
}

// Value of lane (l ^ M) for M in {1, 2, 4, 8}: DPP quad permutes for 1 and 2,
// a swizzle for 4 and a row rotation by 8 (16-lane rows) for 8.
template <int M>
__device__ inline int xor_lane_i32(int x)
{
    static_assert(M == 1 || M == 2 || M == 4 || M == 8, "mask");
    if constexpr (M == 1) return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);
    else if constexpr (M == 2) return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);
    else if constexpr (M == 4) return __builtin_amdgcn_ds_swizzle(x, 0x101F);
    else return __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);
}

template <int M>
__device__ inline double xor_lane_f64(double x)
{
    if constexpr (M >= 16) {
        return __shfl_xor(x, M);
    } else {
        const int lo = xor_lane_i32<M>(__double2loint(x));
        const int hi = xor_lane_i32<M>(__double2hiint(x));
        return __hiloint2double(hi, lo);
    }
}

// Transposing reduction of E per-lane values over the 64 lanes of a wavefront.
// On entry lane l holds v[0..E-1], its partial sums for E different events.
// On return every lane holds the full 64-lane sum of v[j] for
//   j = l / (64 / E),
// i.e. lanes are grouped in runs of 64/E, one run per event.  Each butterfly
// level halves the number of live values by exchanging half of them with the
// partner lane (bit M of the lane index flipped), so E values cost E - 1
// exchanges instead of the 6E of E separate reductions.  The order of
// additions is fixed and every lane of a run adds the same two operands at
// each level, so the result is bit-reproducible and identical across a run.
template <int E, int H, int M>
__device__ inline void transpose_level(double (&v)[E], int lane)
{
    if constexpr (H >= 1) {
        if constexpr (M == 32 || M == 16) {
#pragma unroll
            for (int j = 0; j < H; ++j) {
                if constexpr (M == 32) swap32_f64(v[j], v[j + H]);
                else swap16_f64(v[j], v[j + H]);
                v[j] = v[j] + v[j + H];
            }
        } else {
            const bool up = (lane & M) != 0;
#pragma unroll
            for (int j = 0; j < H; ++j) {
                const double send = up ? v[j] : v[j + H];
                const double keep = up ? v[j + H] : v[j];
                v[j] = keep + xor_lane_f64<M>(send);
            }
        }
        transpose_level<E, H / 2, M / 2>(v, lane);
    }
}

// Sum over the lanes that differ from this one only in bits below 2M
// (M = 32 / E at the first call): a plain butterfly all-reduce.
template <int M>
__device__ inline double allreduce_low(double s)
{
    if constexpr (M >= 1) {
        if constexpr (M == 32) {
            double a = s, b = s;
            swap32_f64(a, b);
            s = a + b;
        } else if constexpr (M == 16) {
            double a = s, b = s;
            swap16_f64(a, b);
            s = a + b;
        } else {
            s = s + xor_lane_f64<M>(s);
        }
        return allreduce_low<M / 2>(s);
    }
    return s;
}

template <int E>
__device__ inline double transpose_reduce(double (&v)[E], int lane)
{
    static_assert(E >= 1 && E <= 64 && (E & (E - 1)) == 0, "E must be a power of two <= 64");
    transpose_level<E, E / 2, 32>(v, lane);
    return allreduce_low<32 / E>(v[0]);
}

// 1/x for finite x > 0: hardware reciprocal estimate refined by two
// Newton-Raphson steps r <- r + r (1 - x r).
__device__ inline double recip_f64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __fma_rn(-x, r, 1.0);
    r = __fma_rn(r, e, r);
    e = __fma_rn(-x, r, 1.0);
    return __fma_rn(r, e, r);
}

// Packed index of (a, b), a <= b, in the row-major upper triangle of W x W.
__host__ __device__ inline int packed_index(int W, int a, int b)
{
    return a * W - (a * (a - 1)) / 2 + (b - a);
}

// Wave-local ordering of LDS traffic: LDS operations of one wavefront are
// processed in order; this keeps the compiler from moving accesses across it.
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace pwa
