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

// Transposing reduction of E per-lane values over the 64 lanes of a wavefront.
// On entry lane l holds v[0..E-1], its partial sums for E different events.
// On return every lane holds the full 64-lane sum of v[j] for
//   j = l / (64 / E),
// i.e. lanes are grouped in runs of 64/E, one run per event.  Each butterfly
// level halves the number of live values by exchanging half of them with the
// partner lane (lane ^ m), so E values cost E - 1 exchanges instead of the
// 6E of E separate reductions.  The order of additions is fixed, so the
// result is bit-reproducible and identical across the lanes of a run.
template <int E, int H, int M>
__device__ inline void transpose_level(double (&v)[E], int lane)
{
    if constexpr (H >= 1) {
        const bool up = (lane & M) != 0;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const double send = up ? v[j] : v[j + H];
            const double keep = up ? v[j + H] : v[j];
            v[j] = keep + __shfl_xor(send, M);
        }
        transpose_level<E, H / 2, M / 2>(v, lane);
    }
}

template <int E>
__device__ inline double transpose_reduce(double (&v)[E], int lane)
{
    static_assert(E >= 1 && E <= 64 && (E & (E - 1)) == 0, "E must be a power of two <= 64");
    transpose_level<E, E / 2, 32>(v, lane);
    double s = v[0];
#pragma unroll
    for (int m = 32 / E; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    return s;
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
