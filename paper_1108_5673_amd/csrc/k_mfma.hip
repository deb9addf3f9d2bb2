// k_mfma.hip -- the amplitude form for many parameter vectors at once, on the
// matrix cores (Eq. 1 and Eq. 3 for K vectors V_1..V_K in one pass).
//
// The fits of Sec. 2 are repeated from many starting points; evaluating K of
// them together turns S_ik = sum_a A_ia V_ak into a matrix product.  In real
// arithmetic each event gives two rows over KD = 2W (padded to 16 NS) columns,
//     x_i  = [Re A_i0, Im A_i0, Re A_i1, Im A_i1, ...],
//     x'_i = [Im A_i0, -Re A_i0, Im A_i1, -Re A_i1, ...],
// and each vector one column b_k = [Re V_0k, -Im V_0k, Re V_1k, -Im V_1k, ...]:
//     Re S_ik = x_i . b_k,   Im S_ik = x'_i . b_k,
// so S is a (2 events x KD) by (KD x K) product whose output holds Re S and
// Im S of one (event, vector) pair in neighbouring rows.  The adjoint needs
// g_bk = sum_i c_ik conj(A_ib) with c_ik = S_ik / I_ik, the product
// G = Y C over the (event, Re/Im) rows with
//     Re g_bk = sum_i Re c_ik Re A_ib + Im c_ik Im A_ib   (row 2b of Y: [Re A_ib | Im A_ib]),
//     Im g_bk = sum_i Im c_ik Re A_ib - Re c_ik Im A_ib   (row 2b + 1: [-Im A_ib | Re A_ib]),
// whose rows are the 2W real gradient components directly.
//
// Both products run on the 32x32x16 16-bit MFMA with FP32 accumulation, over
// tiles of 16 events (32 rows):
//   * forward: A operand = the 32 rows of the tile x 16 of KD (lane l: row
//     l % 32, KD 8 (l / 32) .. + 7), B operand = the vector matrix (lane l:
//     vector l % 32); the accumulator gives lane l vector l % 32 and rows
//     8 j + 4 (l / 32) + i in register 4 j + i, so registers 2 r and 2 r + 1
//     are Re S and Im S of one event (event 4 j + 2 (l / 32) + i / 2);
//   * epilogue in registers, one lane per (event, vector) pair: I = Re^2 + Im^2,
//     ln I, w = 1 / I and c = S w;
//   * adjoint: registers 8 s .. 8 s + 7 of the accumulator are exactly the B
//     operand of an MFMA whose 16 k-slots are the rows 16 s .. 16 s + 15 of the
//     tile; the A operand (lane l: output row l % 32, the same 8 slots) comes
//     from a second copy of the tile stored in that slot order.
//     So S never leaves the registers.  When KD is an odd multiple of 16 the
//     last 16 gradient rows run on the 16x16x32 MFMA instead of a 32-row block
//     that would be half padding: one lane-16 swap of the two halves' weight
//     registers makes them its A operand (16 vectors x 32 slots), the stored
//     rows its B operand.
// Merged last step (bf16, 2W mod 16 in 1..8): the last 16-wide K-step holds
// at most 8 real columns, so its upper 8 slots repeat them (both rows of an
// event) and the first V part's matrix holds there the second part's rows of
// those columns: one MFMA adds both parts of that step, and the second part
// runs NS - 1 steps.
// Scale: each vector enters as V_k / s_k with s_k the power of two nearest
// ||V_k||_2, so S, I and c = S / I stay near unit magnitude whatever the size of
// V (float16 has a narrow exponent range); the assembly undoes it exactly:
// ln I = ln I' + 2 ln s_k and g = g' / s_k.
// Accuracy: the amplitudes are stored in the 16-bit type (the input of this
// form).  V is split into two 16-bit parts (about 16 significant bits for
// bf16, 22 for fp16) whose products are accumulated; the part of V they leave
// out changes every S_i coherently, and its first-order share of sum ln I,
// 2 Re sum_a V_lo,a conj(g_a) (g the adjoint sums the kernel forms anyway), is
// added back in the assembly, so that the parameters, which every event
// shares, add no coherent 16-bit rounding to the NLL.  The weights c are split
// into two parts (see Split below).  Per lane, log2 I of
// the step's eight (event, vector) pairs is taken in FP32 (hardware v_log_f32)
// and summed in FP32, then added to an FP64 lane sum.  The adjoint's FP32
// accumulators add at most kFoldTiles tiles: they are then added into FP64
// sums in LDS (one slot per lane and accumulator register) and restart from
// zero.  All cross-block sums are FP64.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <mutex>
#include <type_traits>
#include <hip/hip_fp16.h>

#include "pwa_internal.h"
#include "tail.h"
#include "wave_ops.h"

namespace pwa {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Splitting a value into 16-bit parts.  bf16 has the exponent range of FP32,
// so its parts (two for V and two for c) are plain successive remainders,
// accumulated together.  fp16 would make the low part subnormal for values
// below about 0.125, and subnormal fp16 inputs do not reliably survive the
// conversion and the matrix product, so an fp16 split keeps every part normal:
// the high part is zero below 2^-14, the low part is stored multiplied by 2^11
// and accumulated on its own, and the two accumulators are recombined exactly.
template <typename T> struct Split;
template <> struct Split<__bf16> {
    static constexpr int kVParts = 2;
    static constexpr bool kScaledLow = false;
};
template <> struct Split<_Float16> {
    static constexpr int kVParts = 2;
    static constexpr bool kScaledLow = true;
};
template <typename T> constexpr int mfma_v_parts() { return Split<T>::kVParts; }
constexpr float kLowScale = 2048.0f;          // 2^11
constexpr float kLowUnscale = 1.0f / 2048.0f;
constexpr float kHalfNormalMin = 6.103515625e-05f;   // 2^-14

template <typename T> struct H16;
template <> struct H16<__bf16> {
    typedef __bf16 V8 __attribute__((ext_vector_type(8)));
    typedef __bf16 V2 __attribute__((ext_vector_type(2)));
    __device__ static f32x16 mfma(V8 a, V8 b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    __device__ static f32x4 mfma16(V8 a, V8 b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct H16<_Float16> {
    typedef _Float16 V8 __attribute__((ext_vector_type(8)));
    typedef _Float16 V2 __attribute__((ext_vector_type(2)));
    __device__ static f32x16 mfma(V8 a, V8 b, f32x16 c)
    {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
    __device__ static f32x4 mfma16(V8 a, V8 b, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// float -> 16-bit, round to nearest even
__device__ inline __bf16 to16(float x, __bf16*) { return (__bf16)x; }
__device__ inline _Float16 to16(float x, _Float16*) { return (_Float16)x; }
template <typename T> __device__ inline T round16(float x) { return to16(x, (T*)nullptr); }

// high part of a two-part split: the rounded value, or zero where fp16 would
// be subnormal
template <typename T> __device__ inline T split_hi(float x)
{
    if constexpr (Split<T>::kScaledLow)
        if (fabsf(x) < kHalfNormalMin) return round16<T>(0.f);
    return round16<T>(x);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two-part split of a pair of values, each part rounded to nearest even by one
// paired conversion.  The high part is the rounded value (zero where fp16 would
// be subnormal); the low part is the remainder, times 2^11 for fp16.
// The remainders x_j - hi_j are exact in FP32 (hi_j is x_j rounded to 8 or 11
// significant bits); each comes from one dot-product instruction of the packed
// high parts with m0 = (-1, 0) or m1 = (0, -1) added to x_j, whose bf16 x bf16
// and f16 x f16 products are exact.  The multipliers must be held in registers
// (make_split_multipliers): written as vector constants, the compiler encodes
// (-1, 0) as the FP32 inline constant -1.0, whose 16-bit halves the
// instruction reads as (0, -1), so the wrong part would be subtracted.
template <typename T> struct SplitMul {
    typename H16<T>::V2 m0, m1;
};
template <typename T> __device__ inline SplitMul<T> make_split_multipliers()
{
    using V2 = typename H16<T>::V2;
    // -1 in the low or the high 16 bits: 0xBF80 (bf16) or 0xBC00 (fp16)
    unsigned lo = Split<T>::kScaledLow ? 0x0000BC00u : 0x0000BF80u;
    unsigned hi = lo << 16;
    asm volatile("" : "+v"(lo), "+v"(hi));   // registers, never inline constants
    return SplitMul<T>{__builtin_bit_cast(V2, lo), __builtin_bit_cast(V2, hi)};
}

template <typename T>
__device__ inline void split_pair(float x0, float x1, const SplitMul<T>& sm,
                                  typename H16<T>::V2& hi, typename H16<T>::V2& lo)
{
    using V2 = typename H16<T>::V2;
    const f32x2 x = {x0, x1};
    if constexpr (Split<T>::kScaledLow) {
        const f32x2 xh = {fabsf(x0) < kHalfNormalMin ? 0.f : x0,
                          fabsf(x1) < kHalfNormalMin ? 0.f : x1};
        hi = __builtin_convertvector(xh, V2);
    } else {
        hi = __builtin_convertvector(x, V2);
    }
    f32x2 r;
    if constexpr (Split<T>::kScaledLow) {
        r[0] = __builtin_amdgcn_fdot2(hi, sm.m0, x0, false) * kLowScale;
        r[1] = __builtin_amdgcn_fdot2(hi, sm.m1, x1, false) * kLowScale;
    } else {
        r[0] = __builtin_amdgcn_fdot2_f32_bf16(hi, sm.m0, x0, false);
        r[1] = __builtin_amdgcn_fdot2_f32_bf16(hi, sm.m1, x1, false);
    }
    lo = __builtin_convertvector(r, V2);
}

// a stored amplitude component: rounded to nearest even; fp16 storage holds
// no subnormals, they are stored as zero (the value the matrix product is
// certain to use)
template <typename T> __device__ inline T store16(float x)
{
    T y = round16<T>(x);
    if constexpr (Split<T>::kScaledLow)
        if (fabsf((float)y) < kHalfNormalMin) y = round16<T>(0.f);
    return y;
}

// Slot of (event e of a tile, part p: 0 Re, 1 Im) in the adjoint operand rows:
// the forward accumulator holds it in register 8 s + u of the lanes with
// l / 32 = h, which the adjoint MFMA of step s reads as k-slot 8 h + u.
__device__ inline int mfma_slot(int e, int p)
{
    const int s = e >> 3, e7 = e & 7;
    const int h = (e7 >> 1) & 1;
    const int u = 4 * (e7 >> 2) + 2 * (e7 & 1) + p;
    return 16 * s + 8 * h + u;
}

// ---- build: the two copies of the event tiles -------------------------------
// Tiles of 16 events; the buffers are zeroed before packing (padding events,
// KD columns beyond 2W and adjoint rows beyond 2W stay zero).
// af: [tile][32 rows][KD]            (forward A operand: rows 2e = x_e, 2e + 1 = x'_e)
// at: [tile][mfma_at_tile_elems(KD)] (adjoint operand rows: row 2b = [Re A_eb | Im A_eb],
//                                     row 2b + 1 = [-Im A_eb | Re A_eb] at slots
//                                     mfma_slot(e, 0 | 1)); rows in full blocks of
//     32 rows x 32 slots (the A operand of the 32x32x16 MFMA, lane l: row l % 32);
//     when KD is an odd multiple of 16 the last 16 rows form one block in the B
//     operand order of the 16x16x32 MFMA: lane l holds row 32 RF + l % 16 at the 8
//     slots of lane group q = l / 16 in the order q -> 16 (q & 1) + 8 (q >> 1) (the
//     order in which one lane-16 swap of the two halves' weights delivers them)
__device__ inline int64_t mfma_at_offset(int KD, int64_t tile, int row, int slot)
{
    const int rf = KD / 32;   // full 32-row blocks
    int64_t o = tile * mfma_at_tile_elems(KD);
    if (row < 32 * rf) return o + (int64_t)row * 32 + slot;
    const int q = (slot >> 4) + 2 * ((slot >> 3) & 1);
    return o + rf * 1024 + (int64_t)((row - 32 * rf) + 16 * q) * 8 + (slot & 7);
}

template <typename T>
__global__ void k_pack_mfma(const void* __restrict__ src, bool c128, int64_t n, int W, int KD,
                            bool merge, T* __restrict__ af, T* __restrict__ at)
{
    const int64_t total = n * (int64_t)W;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ev = g / W;
        const int a = (int)(g % W);
        float re, im;
        if (c128) {
            const double2 v = reinterpret_cast<const double2*>(src)[g];
            re = (float)v.x;
            im = (float)v.y;
        } else {
            const float2 v = reinterpret_cast<const float2*>(src)[g];
            re = v.x;
            im = v.y;
        }
        const T yr = store16<T>(re), yi = store16<T>(im);
        const T nr = round16<T>(-(float)yr), ni = round16<T>(-(float)yi);   // exact
        const int64_t tile = ev / kMfmaTile;
        const int e = (int)(ev % kMfmaTile);
        T* x = af + (tile * 32 + 2 * e) * KD + 2 * a;
        x[0] = yr;
        x[1] = yi;
        x[KD] = yi;
        x[KD + 1] = nr;
        if (merge && 2 * a >= KD - 16) {   // the merged last step's repeated columns
            x[8] = yr;
            x[9] = yi;
            x[KD + 8] = yi;
            x[KD + 9] = nr;
        }
        const int s0 = mfma_slot(e, 0), s1 = mfma_slot(e, 1);
        at[mfma_at_offset(KD, tile, 2 * a, s0)] = yr;
        at[mfma_at_offset(KD, tile, 2 * a, s1)] = yi;
        at[mfma_at_offset(KD, tile, 2 * a + 1, s0)] = ni;
        at[mfma_at_offset(KD, tile, 2 * a + 1, s1)] = yr;
    }
}

// ---- per call: the vector matrix, split into NP 16-bit parts --------------
// part p at vm + p * part_elems, element [((cb * NS + s) * 2 + h) * 32 + c][8]:
// vector 32 cb + c, KD rows 16 s + 8 h .. + 7
// power of two nearest ||V_k||_2 (1 for V_k = 0)
__device__ inline double vector_scale(const double* vk, int W)
{
    double nn = 0.0;
    for (int a = 0; a < 2 * W; ++a) nn += vk[a] * vk[a];
    if (!(nn > 0.0)) return 1.0;
    return ldexp(1.0, (int)rint(0.5 * log2(nn)));
}

// The 16-bit parts of one entry x of the scaled vector matrix (x = Re V_a / s
// or -Im V_a / s) and the remainder they leave out, x minus their sum: bf16
// takes two successive remainders, each rounded to nearest (16 significant
// bits in all); fp16 a high part (zero below 2^-14) and the low part times
// 2^11 (22 bits).  The remainder's share of the NLL is added back in the
// assembly (k_assemble_mfma).
template <typename T> struct VSplit {
    T p[Split<T>::kVParts];
    double rest;
};
template <typename T> __device__ inline VSplit<T> split_v(double x)
{
    VSplit<T> r;
    if constexpr (Split<T>::kScaledLow) {
        const T hi = split_hi<T>((float)x);
        const double d = x - (double)(float)hi;
        const T lo = round16<T>((float)(d * kLowScale));
        r.p[0] = hi;
        r.p[1] = lo;
        r.rest = d - (double)(float)lo * (double)kLowUnscale;
    } else {
#pragma unroll
        for (int q = 0; q < Split<T>::kVParts; ++q) {
            const T y = round16<T>((float)x);
            r.p[q] = y;
            x -= (double)(float)y;
        }
        r.rest = x;
    }
    return r;
}

constexpr int kPrepThreads = 256;

// One block per column k of the vector matrix (32 n_cb columns; those past K
// are zero): V_k is read once (from device or mapped host memory), its scale
// s_k formed, and the column's entries written in the layout the main
// kernel's B operand reads (lane c of half h holds entries 16 s + 8 h ..
// 16 s + 8 h + 7 of step s), one array per part; then the vector's
// assembly values above.
template <typename T>
__global__ __launch_bounds__(kPrepThreads) void k_prep_vmat16(
    const double* __restrict__ v, int K, int W, int NS, int n_cb, bool merge,
    const double2* __restrict__ M, T* __restrict__ vm, double* __restrict__ vprep)
{
    __shared__ double s_v[2 * PWA_MAX_WAVES_MATRIX];
    __shared__ double s_wave[kPrepThreads / 64];
    const int k = blockIdx.x;
    const int cb = k / 32, c = k % 32;
    const bool real = k < K;   // uniform over the block
    const int b = threadIdx.x;
    // the first 16 rows of column b of M, loaded while V arrives
    constexpr int kB = 16;
    double2 x0[kB];
#pragma unroll
    for (int j = 0; j < kB; ++j)
        x0[j] = real && b < W && j < W ? M[j * W + b] : make_double2(0.0, 0.0);
    for (int e = threadIdx.x; e < 2 * W; e += blockDim.x)
        s_v[e] = real ? v[(size_t)k * 2 * W + e] : 0.0;
    __syncthreads();
    const double sk = real ? vector_scale(s_v, W) : 1.0;
    // entry e of the scaled column: Re V_a / s (e = 2a, multiplies Re A_a) or
    // -Im V_a / s (e = 2a + 1, multiplies Im A_a)
    auto entry = [&](int e) {
        if (!real || e >= 2 * W) return 0.0;
        return e % 2 == 0 ? s_v[e] / sk : -s_v[e] / sk;
    };
    const size_t part_elems = (size_t)n_cb * NS * 2 * 32 * 8;
    for (int kd = threadIdx.x; kd < 16 * NS; kd += blockDim.x) {
        const int st = kd / 16, h = (kd / 8) % 2, t = kd % 8;
        const size_t g = ((size_t)((cb * NS + st) * 2 + h) * 32 + c) * 8 + t;
        const VSplit<T> sp = split_v<T>(entry(kd));
#pragma unroll
        for (int p = 0; p < Split<T>::kVParts; ++p) vm[p * part_elems + g] = sp.p[p];
        // merged last step: the first part's upper 8 slots of the last K-step
        // hold the second part of the entries 8 below (their repeated columns)
        if (merge && st == NS - 1 && h == 1) vm[g] = split_v<T>(entry(kd - 8)).p[1];
    }
    if (!real) return;
    // m_b = sum_a V_a M_ab (thread b), rows in order, 16 at a time
    double mr = 0.0, mi = 0.0, mu_part = 0.0;
    if (b < W) {
        for (int a0 = 0; a0 < W; a0 += kB) {
            double2 x[kB];
#pragma unroll
            for (int j = 0; j < kB; ++j)
                x[j] = a0 == 0 ? x0[j]
                               : (a0 + j < W ? M[(a0 + j) * W + b] : make_double2(0.0, 0.0));
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                const int a = a0 + j < W ? a0 + j : 0;
                const double vr = s_v[2 * a], vi = s_v[2 * a + 1];
                mr += vr * x[j].x - vi * x[j].y;
                mi += vr * x[j].y + vi * x[j].x;
            }
        }
        mu_part = s_v[2 * b] * mr + s_v[2 * b + 1] * mi;
    }
    const double mu = block_sum_fixed(mu_part, s_wave);
    double* vp = vprep + (size_t)k * vprep_len(W);
    if (threadIdx.x == 0) {
        vp[0] = sk;
        vp[1] = mu;
    }
    if (b < W) {
        vp[2 + 2 * b] = mr;
        vp[3 + 2 * b] = mi;
    }
    for (int o = threadIdx.x; o < 2 * W; o += blockDim.x) vp[2 + 2 * W + o] = split_v<T>(entry(o)).rest;
}

// ---- the fused forward + epilogue + adjoint kernel -------------------------
// grid (chunks, ceil(n_cb / B)), blocks of B = min(n_cb, mfma_waves) wavefronts:
// wavefront w of a block takes column block cb = B blockIdx.y + w (32 vectors)
// over every event tile of the block's chunk, so the wavefronts of a block
// read the same tiles at about the same time and all but the first find them
// in cache.  Records per (chunk, cb, vector): rec_d = [sum ln I, n_bad] (FP64;
// n_bad counts the vector's lane sums that met a degenerate event, so it is
// non-zero exactly when one did) and rec_g = G[0 .. KD) of the vector (the
// wavefront's FP64 sums rounded to FP32; rows 2b, 2b + 1 are Re g_b and Im g_b).
// Up to 8 wavefronts per block (two per SIMD, at most 256 registers each); the
// wider row lengths (NS > 4) need more registers and run 4 (one per SIMD).
template <int NS> constexpr int mfma_waves() { return NS <= 4 ? 8 : 4; }
// FP64 fold slots per lane: 16 per full 32-row block of the adjoint, and 8
// (two 16-vector blocks of 4) for a last block of 16 rows
template <int NS> constexpr int mfma_fold_regs() { return 16 * (NS / 2) + ((NS & 1) ? 8 : 0); }
// An FP32 adjoint accumulator is folded into FP64 once it has added at least
// kFoldTiles tiles (so never more than kFoldTiles + 1).
constexpr int kFoldTiles = 32;

template <typename T, int NS, int NP, bool MRG>
__global__ __launch_bounds__(64 * mfma_waves<NS>()) void k_amp_mfma(
    const T* __restrict__ af, const T* __restrict__ at, const T* __restrict__ vm,
    int64_t n_events, int64_t n_tiles, int n_cols, int n_cb, int chunks,
    double* __restrict__ rec_d, float* __restrict__ rec_g)
{
    constexpr int KD = 16 * NS;
    constexpr bool REM = (NS & 1) != 0;     // a last adjoint block of 16 rows
    constexpr int RF = NS / 2;              // full 32-row adjoint blocks
    constexpr int RFA = RF > 0 ? RF : 1;    // array extent
    constexpr int AT = mfma_at_tile_elems(KD);
    constexpr int NF = mfma_fold_regs<NS>();
    using V8 = typename H16<T>::V8;
    using V2 = typename H16<T>::V2;

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int h = lane >> 5, c = lane & 31;
    const int cb = (int)(blockDim.x >> 6) * blockIdx.y + wave;
    if (cb >= n_cb) return;   // no barrier follows
    const bool col_active = 32 * cb + c < n_cols;

    const size_t part_elems = (size_t)n_cb * NS * 2 * 32 * 8;
    V8 vp[NP][NS];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int s = 0; s < NS; ++s)
            vp[p][s] = *reinterpret_cast<const V8*>(
                vm + p * part_elems + ((size_t)((cb * NS + s) * 2 + h) * 32 + c) * 8);
    constexpr bool SL = Split<T>::kScaledLow;
    static_assert(!MRG || (!SL && NP == 2), "the merged last step adds two parts in one accumulator");
    const SplitMul<T> smul = make_split_multipliers<T>();
    // adjoint accumulators: g (full blocks, 32 rows x 32 vectors) and gr (the
    // last 16 rows: 16 vectors x 16 rows per block of vectors); gl, grl the
    // scaled low parts of fp16
    f32x16 g[RFA], gl[SL ? RFA : 1];
    f32x4 gr[2], grl[SL ? 2 : 1];
#pragma unroll
    for (int rb = 0; rb < RFA; ++rb) g[rb] = f32x16{};
#pragma unroll
    for (int rb = 0; rb < (SL ? RFA : 1); ++rb) gl[rb] = f32x16{};
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) gr[nb] = f32x4{};
#pragma unroll
    for (int nb = 0; nb < (SL ? 2 : 1); ++nb) grl[nb] = f32x4{};
    double dsum = 0.0;
    // FP64 sums of the adjoint accumulators: slot [wave][j][lane] (j: 16 rb + q
    // for the full blocks, 16 RF + 4 nb + r for the last one), each owned by
    // one lane (no synchronisation needed)
    __shared__ double s_gacc[mfma_waves<NS>() * NF * 64];
    double* gacc = s_gacc + (size_t)wave * NF * 64 + lane;
#pragma unroll
    for (int j = 0; j < NF; ++j) gacc[64 * j] = 0.0;
    int since_fold = 0;   // tiles added to g, gl since they were last folded
    auto fold = [&]() {
        since_fold = 0;
#pragma unroll
        for (int rb = 0; rb < RF; ++rb)
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                float x = g[rb][q];
                if constexpr (SL) x = fmaf(gl[rb][q], kLowUnscale, x);
                // LDS add without a return (the slot is this lane's own)
                __hip_atomic_fetch_add(gacc + 64 * (16 * rb + q), (double)x, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        if constexpr (REM) {
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float x = gr[nb][r];
                    if constexpr (SL) x = fmaf(grl[nb][r], kLowUnscale, x);
                    __hip_atomic_fetch_add(gacc + 64 * (16 * RF + 4 * nb + r), (double)x,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
        }
#pragma unroll
        for (int rb = 0; rb < RFA; ++rb) g[rb] = f32x16{};
#pragma unroll
        for (int rb = 0; rb < (SL ? RFA : 1); ++rb) gl[rb] = f32x16{};
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) gr[nb] = f32x4{};
#pragma unroll
        for (int nb = 0; nb < (SL ? 2 : 1); ++nb) grl[nb] = f32x4{};
    };

    // tile indices fit in 32 bits (the host checks n_tiles); 32-bit scalar
    // indices and 32-bit lane offsets from a scalar tile base keep the
    // address arithmetic off the vector ALU
    const int t0 = (int)((int64_t)blockIdx.x * n_tiles / chunks);
    const int t1 = (int)((int64_t)(blockIdx.x + 1) * n_tiles / chunks);
    // operands of one tile: forward rows (32 rows x KD) and adjoint rows (RF
    // blocks of 32 rows x 32 slots, and the last 16 rows)
    struct OpsA {
        V8 a[NS];
    };
    struct OpsB {
        V8 b[RFA][2];
        V8 br;
    };
    const uint32_t a_off = (uint32_t)(c * KD + 8 * h);
    const uint32_t b_off = (uint32_t)(c * 32 + 8 * h);
    const uint32_t r_off = (uint32_t)(RF * 1024 + lane * 8);
    auto load_a = [&](OpsA& o, int t) {
        const T* ta = af + (int64_t)t * (32 * KD);
#pragma unroll
        for (int s = 0; s < NS; ++s)
            o.a[s] = *reinterpret_cast<const V8*>(ta + (size_t)a_off + 16 * s);
    };
    auto load_b = [&](OpsB& o, int t) {
        const T* tt = at + (int64_t)t * AT;
#pragma unroll
        for (int rb = 0; rb < RF; ++rb)
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2)
                o.b[rb][s2] =
                    *reinterpret_cast<const V8*>(tt + (size_t)b_off + rb * 1024 + 16 * s2);
        if constexpr (REM) o.br = *reinterpret_cast<const V8*>(tt + (size_t)r_off);
    };
    // The last 16 adjoint rows on the 16x16x32 MFMA, once both halves' weights
    // of the tile are formed: D[vector][row] += C^T Y with the weights as the A
    // operand (lane l: vector l % 16 of a block of 16, 8 slots of lane group
    // l / 16).  A lane-16 swap of the two halves' registers turns them (lane
    // (c, h): vector c, slots 16 s2 + 8 h ..) into exactly that: the first
    // register then holds vectors 0..15 and the second vectors 16..31, at slot
    // groups 0, 16, 8, 24 (the order of the stored rows).
    auto swap16 = [](V8& x0, V8& x1) {
        u32x4 a = __builtin_bit_cast(u32x4, x0), b = __builtin_bit_cast(u32x4, x1);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const auto r = __builtin_amdgcn_permlane16_swap(a[d], b[d], false, false);
            a[d] = r[0];
            b[d] = r[1];
        }
        x0 = __builtin_bit_cast(V8, a);
        x1 = __builtin_bit_cast(V8, b);
    };
    auto rem_adj = [&](const OpsB& o, V8 c0, V8 c1, V8 l0, V8 l1) {
        swap16(c0, c1);
        swap16(l0, l1);
        gr[0] = H16<T>::mfma16(c0, o.br, gr[0]);
        gr[1] = H16<T>::mfma16(c1, o.br, gr[1]);
        if constexpr (SL) {
            grl[0] = H16<T>::mfma16(l0, o.br, grl[0]);
            grl[1] = H16<T>::mfma16(l1, o.br, grl[1]);
        } else {
            gr[0] = H16<T>::mfma16(l0, o.br, gr[0]);
            gr[1] = H16<T>::mfma16(l1, o.br, gr[1]);
        }
    };
    // S of the tile's 16 events x 32 vectors
    auto forward = [&](const OpsA& o) {
        f32x16 acc = f32x16{};
        if constexpr (SL) {
            f32x16 acc_lo = f32x16{};
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                acc = H16<T>::mfma(o.a[s], vp[0][s], acc);
                acc_lo = H16<T>::mfma(o.a[s], vp[1][s], acc_lo);
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] = fmaf(acc_lo[q], kLowUnscale, acc[q]);
        } else {
#pragma unroll
            for (int p = NP - 1; p >= 0; --p)   // smallest parts first
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    if (MRG && p == 1 && s == NS - 1) continue;   // in part 0's last step
                    acc = H16<T>::mfma(o.a[s], vp[p][s], acc);
                }
        }
        return acc;
    };
    auto finish = [&](const f32x16& acc, const OpsB& o, int t, auto fast_tag) {
        constexpr bool fast = decltype(fast_tag)::value;
        // Epilogue and adjoint, in two halves of 8 registers (the adjoint MFMA
        // of half s2 takes registers 8 s2 .. 8 s2 + 7).  Registers (q, q + 1),
        // q even, are Re S and Im S of event 4 (q / 4) + 2 h + (q / 2) % 2 of
        // the tile.  A full tile whose columns all carry vectors needs no
        // validity test: a degenerate event (I not positive and finite) only
        // has to be counted (its NLL is +inf whatever the sum, and its weight
        // 0 * inf or x * NaN is NaN); the last tile and the padding columns
        // take the general path.
        const int nvalid = (int)min<int64_t>(kMfmaTile, n_events - (int64_t)t * kMfmaTile);
        float lsum = 0.f;
        V8 chis[2], clos[2];
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
            V8 chi, clo;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int q = 8 * s2 + 2 * r;
                const float x = acc[q], y = acc[q + 1];
                const float I = fmaf(y, y, x * x);
                const float w = __builtin_amdgcn_rcpf(I);
                float cr, ci;
                // a degenerate I (0, negative, inf or NaN) makes log2 I and so
                // this lane's sum non-finite: that is how it is detected
                if constexpr (fast) {
                    cr = x * w;
                    ci = y * w;
                    lsum += __builtin_amdgcn_logf(I);
                } else {
                    const int e = 4 * (q >> 2) + 2 * h + ((q >> 1) & 1);
                    const bool valid = col_active && e < nvalid;
                    // positive normal or subnormal: not 0, negative, inf or NaN
                    const bool ok = __builtin_amdgcn_classf(I, 0x180);
                    cr = valid ? (ok ? x * w : NAN) : 0.f;
                    ci = valid ? (ok ? y * w : NAN) : 0.f;
                    lsum += valid ? __builtin_amdgcn_logf(I) : 0.f;
                }
                V2 hi, lo;
                split_pair<T>(cr, ci, smul, hi, lo);
                chi[2 * r] = hi[0];
                chi[2 * r + 1] = hi[1];
                clo[2 * r] = lo[0];
                clo[2 * r + 1] = lo[1];
            }
#pragma unroll
            for (int rb = 0; rb < RF; ++rb) {
                g[rb] = H16<T>::mfma(o.b[rb][s2], chi, g[rb]);
                if constexpr (SL) gl[rb] = H16<T>::mfma(o.b[rb][s2], clo, gl[rb]);
                else g[rb] = H16<T>::mfma(o.b[rb][s2], clo, g[rb]);
            }
            chis[s2] = chi;
            clos[s2] = clo;
        }
        if constexpr (REM) rem_adj(o, chis[0], chis[1], clos[0], clos[1]);
        dsum += (double)lsum * 0.69314718055994530942;   // log2 -> ln
    };

    // ---- full tiles, software-pipelined --------------------------------------
    // One step takes the epilogue and adjoint of tile t and the forward product
    // of tile t + 1, in 8 pieces fenced against reordering: piece i holds the
    // epilogue of one register pair (one (event, vector) pair of half i / 4)
    // beside a share of the forward MFMAs, and pieces 4..7 also the adjoint
    // MFMAs of half 0.  The wavefront issues each piece's vector instructions
    // while its MFMAs run.
    constexpr int kFwd = SL ? 2 * NS : NS * NP - (MRG ? 1 : 0);
    auto fwd_mfma = [&](const OpsA& an, f32x16& nx, f32x16& nxl, int m) {
        if constexpr (SL) {
            const int s = m >> 1;
            if (m & 1) nxl = H16<T>::mfma(an.a[s], vp[1][s], nxl);
            else nx = H16<T>::mfma(an.a[s], vp[0][s], nx);
        } else if constexpr (MRG) {
            // part 1 over its first NS - 1 steps, then part 0 over all NS
            if (m < NS - 1) nx = H16<T>::mfma(an.a[m], vp[1][m], nx);
            else nx = H16<T>::mfma(an.a[m - (NS - 1)], vp[0][m - (NS - 1)], nx);
        } else {
            const int p = NP - 1 - m / NS, s = m % NS;   // smallest parts first
            nx = H16<T>::mfma(an.a[s], vp[p][s], nx);
        }
    };
    auto adj_mfma = [&](const OpsB& o, const V8& chi, const V8& clo, int s2, int j) {
        const int rb = j >> 1;
        if (j & 1) {
            if constexpr (SL) gl[rb] = H16<T>::mfma(o.b[rb][s2], clo, gl[rb]);
            else g[rb] = H16<T>::mfma(o.b[rb][s2], clo, g[rb]);
        } else {
            g[rb] = H16<T>::mfma(o.b[rb][s2], chi, g[rb]);
        }
    };
    // One (event, vector) pair of the step's epilogue: I, the weights split
    // into 16-bit parts; returns I.  The logarithms are taken per product of
    // four intensities (see step).
    auto pair_epi = [&](const f32x16& acc, int q, V8& chi, V8& clo, int r) {
        const float x = acc[q], y = acc[q + 1];
        const float I = fmaf(y, y, x * x);
        const float w = __builtin_amdgcn_rcpf(I);
        V2 hi, lo;
        split_pair<T>(x * w, y * w, smul, hi, lo);
        chi[2 * r] = hi[0];
        chi[2 * r + 1] = hi[1];
        clo[2 * r] = lo[0];
        clo[2 * r + 1] = lo[1];
        return I;
    };
    // sum_i log2 I_i of a step: log2 of the products of pairs 0-3 and 4-7, each
    // one FP32 logarithm.  When a product is not a positive normal number (an
    // intensity far from 1 under- or overflowed it, or an event is degenerate)
    // in some lane, the wavefront takes the eight logarithms instead; a
    // degenerate I then makes the sum non-finite, which is how it is counted.
    auto step = [&](const OpsA& an, const f32x16& acc, const OpsB& o) {
        f32x16 nx = f32x16{}, nxl = f32x16{};
        float I[8];
        float p0 = 1.f, p1 = 1.f, l0 = 0.f, l1 = 0.f;
        V8 chi0, clo0, chi1, clo1;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
#pragma unroll
            for (int m = i * kFwd / 8; m < (i + 1) * kFwd / 8; ++m) fwd_mfma(an, nx, nxl, m);
            if (i >= 4) {
#pragma unroll
                for (int j = (i - 4) * 2 * RF / 4; j < (i - 3) * 2 * RF / 4; ++j)
                    adj_mfma(o, chi0, clo0, 0, j);
            }
            if (i < 4) {
                I[i] = pair_epi(acc, 2 * i, chi0, clo0, i);
                p0 *= I[i];
            } else {
                I[i] = pair_epi(acc, 8 + 2 * (i - 4), chi1, clo1, i - 4);
                p1 *= I[i];
            }
            if (i == 3) {
                l0 = __builtin_amdgcn_logf(p0);
                asm volatile("" : "+v"(l0));   // keep the logarithm in this piece
            }
            if (i == 7) {
                l1 = __builtin_amdgcn_logf(p1);
                asm volatile("" : "+v"(l1));
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int j = 0; j < 2 * RF; ++j) adj_mfma(o, chi1, clo1, 1, j);
        if constexpr (REM) rem_adj(o, chi0, chi1, clo0, clo1);
        float lsum = l0 + l1;
        // positive normal: class bit 8
        if (!(__builtin_amdgcn_classf(p0, 0x100) && __builtin_amdgcn_classf(p1, 0x100))) {
            lsum = 0.f;
#pragma unroll
            for (int i = 0; i < 8; ++i) lsum += __builtin_amdgcn_logf(I[i]);
        }
        dsum += (double)lsum * 0.69314718055994530942;   // log2 -> ln
        if constexpr (SL) {
#pragma unroll
            for (int q = 0; q < 16; ++q) nx[q] = fmaf(nxl[q], kLowUnscale, nx[q]);
        }
        return nx;
    };

    // Full tiles: below the last one, when every column carries a vector (no
    // validity tests: a degenerate event makes the lane's log sum non-finite).
    // Operands are loaded a step ahead; loads and products past the last full
    // tile repeat that tile and are not used.
    const int t_full = 32 * cb + 32 <= n_cols ? (int)(n_events / kMfmaTile) : 0;
    const int tf = max(t0, min(t1, t_full));
    int t = t0;
    if (tf - t0 >= 2) {
        OpsA a0, a1;
        OpsB b0, b1;
        load_a(a0, t0);
        load_b(b0, t0);
        load_a(a1, t0 + 1);
        f32x16 s0 = forward(a0);
        // at the top: s0 = S(t), b0 = adjoint operands of t, a1 = forward
        // operands of t + 1 (a0 and b1 free)
        for (; t + 2 <= tf; t += 2) {
            load_a(a0, min(t + 2, tf - 1));
            load_b(b1, t + 1);
            const f32x16 s1 = step(a1, s0, b0);
            load_a(a1, min(t + 3, tf - 1));
            load_b(b0, min(t + 2, tf - 1));
            s0 = step(a0, s1, b1);
            since_fold += 2;
            if (since_fold >= kFoldTiles) fold();
        }
        if (t < tf) {   // an odd count: s0, b0 hold the last full tile
            finish(s0, b0, t, std::true_type{});
            ++t;
            ++since_fold;
        }
    }
    // the rest (a chunk with fewer than two full tiles, the last tile, padded
    // columns): one tile at a time, the next tile's operands loaded ahead
    auto run = [&](const OpsA& oa, const OpsB& ob, int tt) {
        if (tt < t_full) finish(forward(oa), ob, tt, std::true_type{});
        else finish(forward(oa), ob, tt, std::false_type{});
    };
    if (t < t1) {
        OpsA a0, a1;
        OpsB b0, b1;
        load_a(a0, t);
        load_b(b0, t);
        for (; t < t1; t += 2) {
            if (t + 1 < t1) {
                load_a(a1, t + 1);
                load_b(b1, t + 1);
            }
            run(a0, b0, t);
            if (t + 1 < t1) {
                if (t + 2 < t1) {
                    load_a(a0, t + 2);
                    load_b(b0, t + 2);
                }
                run(a1, b1, t + 1);
            }
            since_fold += t + 1 < t1 ? 2 : 1;
            if (since_fold >= kFoldTiles) fold();
        }
    }
    fold();   // the FP64 sums now hold everything; the accumulators are zero
    // records of this wavefront: G column c (vector 32 cb + c), rows
    // 8 j + 4 h + i of each full row block; of the last 16 rows, row
    // 32 RF + l % 16 of vectors 16 nb + 4 (l / 16) + r; and the vector's sum
    // ln I (lanes c and c + 32)
    const size_t rec0 = ((size_t)blockIdx.x * n_cb + cb) * 32;
    const size_t rec_idx = rec0 + c;
    float* gcol = rec_g + rec_idx * KD;
#pragma unroll
    for (int rb = 0; rb < RF; ++rb)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int r = rb * 32 + 8 * (q >> 2) + 4 * h + (q & 3);
            gcol[r] = (float)gacc[64 * (16 * rb + q)];
        }
    if constexpr (REM) {
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int vec = 16 * nb + 4 * (lane >> 4) + r;
                rec_g[(rec0 + vec) * KD + 32 * RF + (lane & 15)] =
                    (float)gacc[64 * (16 * RF + 4 * nb + r)];
            }
    }
    const double other = __shfl_xor(dsum, 32);
    if (h == 0) {
        rec_d[2 * rec_idx] = dsum + other;
        rec_d[2 * rec_idx + 1] = (isfinite(dsum) ? 0.0 : 1.0) + (isfinite(other) ? 0.0 : 1.0);
    }
}

// ---- assembly: one block per vector k ---------------------------------------
struct BatchTail {
    const double* rec_d;   // chunks x n_cb x 32 x 2
    const float* rec_g;    // chunks x n_cb x 32 x KD
    int chunks, n_cb, KD, W, K;
    int64_t n_events;
    const double* vprep;   // K x vprep_len(W) per-vector values (device)
    double* out;           // K x (2 + 2W) (pinned host memory, or device memory)
    unsigned long long* done;   // K completion words (pinned host memory), or null
    unsigned long long seq;
};

constexpr int kBatchAsmThreads = 256;

// One block per vector k.  Every loop issues its loads in batches before
// using them (a loop that adds each value as it arrives waits one memory round
// trip per value).
template <typename T>
__global__ __launch_bounds__(kBatchAsmThreads) void k_assemble_mfma(BatchTail bt)
{
    __shared__ double s_wave[kBatchAsmThreads / 64];
    __shared__ double s_part[kBatchAsmThreads];
    const int k = blockIdx.x;
    const int W = bt.W;
    const int cb = k / 32, c0 = k % 32;
    const double* vp = bt.vprep + (size_t)k * vprep_len(W);
    auto ridx = [&](int ch, int cc) { return ((size_t)ch * bt.n_cb + cb) * 32 + cc; };
    // sum ln I and n_bad over chunks
    double d = 0.0, nb = 0.0;
    for (int ch = threadIdx.x; ch < bt.chunks; ch += blockDim.x) {
        const double2 p0 = *reinterpret_cast<const double2*>(bt.rec_d + 2 * ridx(ch, c0));
        d += p0.x;
        nb += p0.y;
    }
    // gradient records: output o = 2 b + part (G row o: Re g_b, Im g_b) over R
    // chunk ranges (thread o + 2W r takes chunks r, r + R, ... in order; the R
    // partial sums are added in order at the end), loaded in batches of 48
    const int nout = 2 * W;
    const int R = kBatchAsmThreads / nout;
    const int o = threadIdx.x % nout, r = threadIdx.x / nout;
    double m = 0.0, rest = 0.0;
    if (threadIdx.x < nout) {
        m = vp[2 + threadIdx.x];
        rest = vp[2 + nout + threadIdx.x];
    }
    if (r < R) {
        // component o of this vector's record of chunk ch: gk[ch * cstride]
        // (the records of all chunks hold fewer than 2^31 values)
        const float* gk = bt.rec_g + ridx(0, c0) * bt.KD + o;
        const int cstride = bt.n_cb * 32 * bt.KD;
        double x = 0.0;
        constexpr int kB = 48;
        for (int ch0 = r; ch0 < bt.chunks; ch0 += kB * R) {
            // every load is issued (a chunk past the last reads the last and
            // is not added), so that none sits behind a branch that waits
            float u[kB];
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                const int ch = min(ch0 + j * R, bt.chunks - 1);
                u[j] = gk[ch * cstride];
            }
#pragma unroll
            for (int j = 0; j < kB; ++j)
                if (ch0 + j * R < bt.chunks) x += (double)u[j];
        }
        s_part[threadIdx.x] = x;
    }
    const double sk = vp[0];
    const double mu = vp[1];
    const double dsum = block_sum_fixed(d, s_wave) + 2.0 * (double)bt.n_events * log(sk);
    const double nbad = block_sum_fixed(nb, s_wave);   // also orders s_part
    // Component o of the scaled adjoint sums, g'_o (rows 2b, 2b + 1: Re, Im
    // g'_b with g' = s g), and the first-order share of the part of V the
    // split leaves out: with S' computed from V' - V'_lo, sum ln I' is low by
    // 2 Re sum_b V'_lo,b conj(g'_b) (ln |S' + d|^2 = ln |S'|^2 + 2 Re(d / S') +
    // O(d^2), and sum_i A_ib / S'_i = conj(g'_b)).  Entry o of the vector
    // matrix is Re V'_b (o even) or -Im V'_b (o odd).
    double corr = 0.0;
    if (threadIdx.x < nout) {
        double x = 0.0;
        for (int rr = 0; rr < R; ++rr) x += s_part[rr * nout + threadIdx.x];
        const int part = threadIdx.x % 2;
        corr = 2.0 * (part == 0 ? rest : -rest) * x;
        x /= sk;
        store_system(bt.out + (size_t)k * (2 + 2 * W) + 2 + threadIdx.x, 2.0 * (m - x));
    }
    const double dcorr = block_sum_fixed(corr, s_wave);
    if (threadIdx.x == 0) {
        store_system(bt.out + (size_t)k * (2 + 2 * W),
                     nbad > 0.0 ? INFINITY : (-(dsum + dcorr) + mu));
        store_system(bt.out + (size_t)k * (2 + 2 * W) + 1, nbad);
    }
    if (!bt.done) return;   // results in device memory, stream-ordered: nothing to publish
    wait_vm_complete();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(bt.done + k, bt.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ---- launchers --------------------------------------------------------------
static int grid_for(int64_t total, int block)
{
    int64_t g = (total + block - 1) / block;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_pack_mfma(const void* src, bool c128, int64_t n, int W, bool bf,
                            const Model& m, hipStream_t s)
{
    const int64_t total = n * (int64_t)W;
    if (bf)
        hipLaunchKernelGGL(k_pack_mfma<__bf16>, dim3(grid_for(total, 256)), dim3(256), 0, s, src,
                           c128, n, W, m.kd, m.fwd_merge, (__bf16*)m.d_data, (__bf16*)m.d_at);
    else
        hipLaunchKernelGGL(k_pack_mfma<_Float16>, dim3(grid_for(total, 256)), dim3(256), 0, s,
                           src, c128, n, W, m.kd, false, (_Float16*)m.d_data, (_Float16*)m.d_at);
    return hipGetLastError();
}

// chunks: about 2048 wavefronts in all (two per SIMD), each with at least a
// few tiles
int mfma_chunks(const Model& m, int n_cb)
{
    int64_t c = (2048 + n_cb - 1) / n_cb;
    const int64_t cap = (m.n_tiles + 3) / 4;
    if (c > cap) c = cap;
    return (int)(c < 1 ? 1 : c);
}

template <typename T, int NS>
static void launch_main(const Model& m, const MfmaBatch& b, hipStream_t s, const LaunchEvents& ev)
{
    constexpr int NP = mfma_v_parts<T>();
    const int wpb = b.n_cb < mfma_waves<NS>() ? b.n_cb : mfma_waves<NS>();
    const int gy = (b.n_cb + wpb - 1) / wpb;
    if constexpr (!Split<T>::kScaledLow) {
        if (m.fwd_merge) {
            hipExtLaunchKernelGGL((k_amp_mfma<T, NS, NP, true>), dim3(b.chunks, gy),
                                  dim3(64 * wpb), 0, s, ev.start, ev.stop, 0, (const T*)m.d_data,
                                  (const T*)m.d_at, (const T*)b.vm, m.n, m.n_tiles, b.K, b.n_cb,
                                  b.chunks, b.rec_d, b.rec_g);
            return;
        }
    }
    hipExtLaunchKernelGGL((k_amp_mfma<T, NS, NP, false>), dim3(b.chunks, gy), dim3(64 * wpb), 0,
                          s, ev.start, ev.stop, 0, (const T*)m.d_data, (const T*)m.d_at,
                          (const T*)b.vm, m.n, m.n_tiles, b.K, b.n_cb, b.chunks, b.rec_d,
                          b.rec_g);
}

template <typename T>
static hipError_t dispatch_ns(const Model& m, const MfmaBatch& b, hipStream_t s,
                              const LaunchEvents& ev)
{
    switch (m.kd / 16) {
    case 1: launch_main<T, 1>(m, b, s, ev); break;
    case 2: launch_main<T, 2>(m, b, s, ev); break;
    case 3: launch_main<T, 3>(m, b, s, ev); break;
    case 4: launch_main<T, 4>(m, b, s, ev); break;
    case 5: launch_main<T, 5>(m, b, s, ev); break;
    case 6: launch_main<T, 6>(m, b, s, ev); break;
    case 7: launch_main<T, 7>(m, b, s, ev); break;
    case 8: launch_main<T, 8>(m, b, s, ev); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t run_batch(const Model& m, const MfmaBatch& b, hipStream_t s,
                            const LaunchEvents& ev)
{
    const int NS = m.kd / 16;
    if (m.n_tiles > INT32_MAX) return hipErrorInvalidValue;   // 32-bit tile indices
    hipLaunchKernelGGL(k_prep_vmat16<T>, dim3(32 * b.n_cb), dim3(kPrepThreads), 0, s, b.v, b.K,
                       m.W, NS, b.n_cb, m.fwd_merge, (const double2*)m.d_M, (T*)b.vm,
                       b.vprep);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return dispatch_ns<T>(m, b, s, ev);
}

size_t mfma_vm_bytes(const Model& m, int n_cb)
{
    const size_t part = (size_t)n_cb * (m.kd / 16) * 2 * 32 * 8 * 2;
    return part * (m.form == kAmpBF16 ? mfma_v_parts<__bf16>() : mfma_v_parts<_Float16>());
}

hipError_t launch_mfma_batch(const Model& m, const MfmaBatch& b, hipStream_t s,
                             const LaunchEvents& ev)
{
    hipError_t e = m.form == kAmpBF16 ? run_batch<__bf16>(m, b, s, ev)
                                      : run_batch<_Float16>(m, b, s, ev);
    if (e != hipSuccess) return e;
    BatchTail bt;
    bt.rec_d = b.rec_d;
    bt.rec_g = b.rec_g;
    bt.chunks = b.chunks;
    bt.n_cb = b.n_cb;
    bt.KD = m.kd;
    bt.W = m.W;
    bt.K = b.K;
    bt.vprep = b.vprep;
    bt.n_events = m.n;
    bt.out = b.out;
    bt.done = b.done;
    bt.seq = b.seq;
    if (m.form == kAmpBF16)
        hipLaunchKernelGGL(k_assemble_mfma<__bf16>, dim3(b.K), dim3(kBatchAsmThreads), 0, s, bt);
    else
        hipLaunchKernelGGL(k_assemble_mfma<_Float16>, dim3(b.K), dim3(kBatchAsmThreads), 0, s, bt);
    return hipGetLastError();
}

// ---- the allocation-free variant: scratch in a static device array --------
// pwa_nll_batched_noalloc keeps the split vector matrix, the vector scales and
// the per-(chunk, column) records in `scratch`, one copy per device, held until
// the process ends.  Host code never passes the array's name to a kernel (on
// the host it names a stand-in, not device memory): the address comes from
// hipGetSymbolAddress, looked up once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(int device, void** out)
{
    static std::mutex mu;
    static void* addr[kNoAllocMaxDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

// Layout of one call's buffers in `scratch` (256-byte aligned pieces): the K
// vector scales, the split vector matrix, then the records of `chunks` event
// chunks; chunks as for pwa_nll_batched when that fits, else fewer.  Returns
// false when not even one chunk fits.
bool noalloc_layout(const Model& m, int K, NoAllocLayout* L)
{
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const int n_cb = (K + 31) / 32;
    const size_t head = up(sizeof(double) * vprep_len(m.W) * (size_t)K) + up(mfma_vm_bytes(m, n_cb));
    const size_t per_chunk = (size_t)n_cb * 32 * (2 * sizeof(double) + sizeof(float) * m.kd);
    if (head + per_chunk > kNoAllocScratchBytes) return false;
    int chunks = mfma_chunks(m, n_cb);
    const size_t fit = (kNoAllocScratchBytes - head) / per_chunk;
    if ((size_t)chunks > fit) chunks = (int)fit;
    L->n_cb = n_cb;
    L->chunks = chunks;
    L->vprep_off = 0;
    L->vm_off = up(sizeof(double) * vprep_len(m.W) * (size_t)K);
    L->rec_d_off = head;
    L->rec_g_off = head + up((size_t)chunks * n_cb * 32 * 2 * sizeof(double));
    return L->rec_g_off + (size_t)chunks * n_cb * 32 * sizeof(float) * m.kd <=
           kNoAllocScratchBytes;
}

// copy of the stored 16-bit amplitudes, widened to complex64 (N x W), read
// from the rows x_i of the forward copy
__global__ void k_unpack_mfma(const void* __restrict__ af, bool bf, int64_t n, int W, int KD,
                              float2* __restrict__ dst)
{
    const int64_t total = n * W;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = g / W;
        const int a = (int)(g % W);
        const int64_t x = ((i / kMfmaTile) * 32 + 2 * (i % kMfmaTile)) * KD + 2 * a;
        float re, im;
        if (bf) {
            re = (float)reinterpret_cast<const __bf16*>(af)[x];
            im = (float)reinterpret_cast<const __bf16*>(af)[x + 1];
        } else {
            re = (float)reinterpret_cast<const _Float16*>(af)[x];
            im = (float)reinterpret_cast<const _Float16*>(af)[x + 1];
        }
        dst[g] = make_float2(re, im);
    }
}

hipError_t launch_unpack_mfma(const Model& m, float* dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_unpack_mfma, dim3(grid_for(m.n * m.W, 256)), dim3(256), 0, s, m.d_data,
                       m.form == kAmpBF16, m.n, m.W, m.kd, (float2*)dst);
    return hipGetLastError();
}

}  // namespace pwa
