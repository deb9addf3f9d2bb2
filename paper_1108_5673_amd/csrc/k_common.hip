// k_common.hip -- the MC integral matrix and the fixed-order final reduction.
//
// M_aa' = (1/N_gen) sum_{j accepted} B_ja B*_ja' (Eq. 3, inner bracket) is built
// once per model in FP64.  Each evaluation ends with one small kernel that
// sums the streaming kernel's per-block records in a fixed order and
// assembles NLL = -sum ln I + mu and G_b = 2 sum_a V_a (M_ab - U_ab) (records
// of packed U: the table forms) or 2 sum_a V_a M_ab - 2 g_b (records of g_b:
// the amplitude form), with mu = sum_a sum_b V_a V*_b M_ab: the MC quadratic
// form is evaluated here, in FP64, once per evaluation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>
#include <utility>

#include "pwa_internal.h"
#include "tail.h"
#include "wave_ops.h"

namespace pwa {

// ---- the MC integral: sum_j B_ja conj(B_jb) over accepted events ---------
// Always on the FP64 matrix cores (below); k_colsum sums the block records.
constexpr int kGramMaxRows = 512;      // partial records of the MC matrix build
constexpr int kGramMfmaMaxTiles = 16;  // matrix-core build for 2W <= 256
constexpr int kGramDepth = 8;          // steps of loads in flight per wavefront

// ---- the MC integral on the FP64 matrix cores (2W <= 256) -----------------
// The real Gram matrix G = sum_j x_j x_j^T of x_j = [Re B_j0 .. Re B_j,W-1,
// Im B_j0 .. Im B_j,W-1] (padded to 16 T; the padding rows and columns of G
// are never read) holds the Hermitian sum:
//   sum_j B_ja conj(B_jb) = G[a][b] + G[W+a][W+b] + i (G[W+a][b] - G[a][W+b]).
// G is a product with the events as its inner dimension, on
// v_mfma_f64_16x16x4f64 (D += A B with A 16 x 4, B 4 x 16): tile pair
// (t <= u) accumulates D[i][j] = sum_k x_k[16 t + i] x_k[16 u + j] over steps
// of 4 events.  Lane l takes event k = l / 16 of the step and component
// i = l % 16 of every tile, which is where both operands expect x_k[16 t + i]
// (A[i][k] and B[k][j] in lane i + 16 k; D[4 r + l / 16][l % 16] in register
// r).  Up to 4 tiles (k_gram_mfma), every tile pair fits one wavefront: the
// four wavefronts of a block take every fourth step of the block's range,
// with the values of the next kGramDepth steps in flight (the memory latency
// is several steps of matrix work), and are added in wavefront order through
// LDS into one record of T (T + 1) / 2 tiles of 256 doubles, in
// register-major order [tile][r][lane].  Wider rows: k_gram_mfma_lds below.
typedef double gd4 __attribute__((ext_vector_type(4)));

template <bool C128, int T>
__global__ __launch_bounds__(256) void k_gram_mfma(const void* __restrict__ mc, int64_t n_acc,
                                                   int W, double* __restrict__ records)
{
    constexpr int NPAIR = T * (T + 1) / 2;
    using In = typename std::conditional<C128, double2, float2>::type;
    using R = typename std::conditional<C128, double, float>::type;   // one real component
    const In* src = reinterpret_cast<const In*>(mc);
    const R* srcr = reinterpret_cast<const R*>(mc);
    __shared__ double s_acc[NPAIR * 4 * 64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i = lane & 15, k = lane >> 4;
    gd4 d[NPAIR];
#pragma unroll
    for (int p = 0; p < NPAIR; ++p) d[p] = gd4{0.0, 0.0, 0.0, 0.0};

    const int64_t n_steps = (n_acc + 3) / 4;
    const int64_t s0 = (int64_t)blockIdx.x * n_steps / gridDim.x;
    const int64_t s1 = (int64_t)(blockIdx.x + 1) * n_steps / gridDim.x;
    // Steps whose four events all exist: component 16 t + i of this lane's
    // event is the real value off[t] places after the step's first event
    // (Re B_c at 2 (k W + c), Im B_c at 2 (k W + c) + 1), read from a scalar
    // step base with a 32-bit lane offset.  The padding components (16 t + i
    // >= 2W) read component 0 instead: they only reach the Gram rows and
    // columns beyond 2W, which the expansion never reads.
    uint32_t off[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int c = 16 * t + i;
        const int cc = c < 2 * W ? c : 0;
        off[t] = (uint32_t)(2 * (k * W + (cc < W ? cc : cc - W)) + (cc < W ? 0 : 1));
    }
    auto load_full = [&](double (&x)[T], int64_t st) {
        const R* base = srcr + st * (int64_t)(8 * W);
#pragma unroll
        for (int t = 0; t < T; ++t) x[t] = (double)base[(size_t)off[t]];
    };
    // any step: events beyond the data, and the padding components, give 0
    auto load_checked = [&](double (&x)[T], int64_t st) {
        const int64_t j = 4 * st + k;
        const bool ev_ok = j < n_acc;
        const int64_t jj = ev_ok ? j : 0;
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int c = 16 * t + i;
            const int cc = c < 2 * W ? c : 0;
            const In b = src[jj * W + (cc < W ? cc : cc - W)];
            const double keep = ev_ok && c < 2 * W ? 1.0 : 0.0;
            x[t] = (double)(cc < W ? b.x : b.y) * keep;
        }
    };
    auto accumulate = [&](const double (&x)[T]) {
        int p = 0;
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int u = t; u < T; ++u, ++p)
                d[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t], x[u], d[p], 0, 0, 0);
    };
    // this wavefront's full steps: first, first + 4, ... below s_full,
    // kGramDepth per trip, each slot of the register ring refilled kGramDepth
    // steps ahead as soon as it is used (refills past the last full step
    // repeat it and are not added)
    const int64_t s_full = min(s1, n_acc / 4);
    const int64_t first = s0 + wave;
    const int64_t n_my = first < s_full ? (s_full - first + 3) / 4 : 0;
    if (n_my > 0) {
        const int64_t last = s_full - 1;
        double xs[kGramDepth][T];
#pragma unroll
        for (int q = 0; q < kGramDepth; ++q) load_full(xs[q], min(first + 4 * q, last));
        for (int64_t q0 = 0; q0 < n_my; q0 += kGramDepth) {
#pragma unroll
            for (int q = 0; q < kGramDepth; ++q) {
                if (q0 + q < n_my) accumulate(xs[q]);
                load_full(xs[q], min(first + 4 * (q0 + q + kGramDepth), last));
            }
        }
    }
    // the step with fewer than four events (only in the last block's range)
    for (int64_t st = s_full; st < s1; ++st) {
        if ((st - s0) % 4 == wave) {
            double x[T];
            load_checked(x, st);
            accumulate(x);
        }
    }

    // the four wavefronts in order, then the block's record
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int p = 0; p < NPAIR; ++p)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int e = (p * 4 + r) * 64 + lane;
                    s_acc[e] = w == 0 ? d[p][r] : s_acc[e] + d[p][r];
                }
        }
        __syncthreads();
    }
    double* rec = records + (int64_t)blockIdx.x * NPAIR * 256;
    for (int e = threadIdx.x; e < NPAIR * 256; e += blockDim.x) rec[e] = s_acc[e];
}

// Wider rows (5 to 16 tiles, 2W <= 256): the tile pairs no longer fit one
// wavefront's registers, so each of the block's NW wavefronts owns a fixed
// range of pairs (at most 9: NW = 4 up to 8 tiles, 16 beyond) and runs over
// every step of the block's range.  The events are staged through LDS in
// chunks of kGramLdsEvents (one row of 16 T doubles per event,
// [Re B | Im B | 0]), loaded once per block with contiguous loads, the next
// chunk's in flight while one is used; each wavefront reads its tiles' values
// from LDS.  Every pair has one owner, which writes its tiles straight into
// the block's record.
constexpr int kGramLdsEvents = 32;

template <int T> constexpr int gram_lds_waves() { return T <= 8 ? 4 : 16; }

// f(std::integral_constant<int, w>{}) for the wavefront index w (uniform), so
// that every pair index in f is a compile-time constant
template <int NW, typename F, int... I>
__device__ inline void for_wave(int wave, F&& f, std::integer_sequence<int, I...>)
{
    ((wave == I ? (f(std::integral_constant<int, I>{}), 0) : 0), ...);
}

template <bool C128, int T, int NW>
__global__ __launch_bounds__(64 * NW, NW == 4 ? 2 : 1) void k_gram_mfma_lds(
    const void* __restrict__ mc, int64_t n_acc, int W, double* __restrict__ records)
{
    constexpr int NT = 64 * NW;                        // threads
    constexpr int NPAIR = T * (T + 1) / 2;
    constexpr int PPW = (NPAIR + NW - 1) / NW;         // pairs per wavefront
    constexpr int XW = 16 * T;                         // LDS row (doubles)
    constexpr int E = kGramLdsEvents;
    constexpr int PRE = (E * 8 * T + NT - 1) / NT;     // staged elements per thread (W <= 8 T)
    using In = typename std::conditional<C128, double2, float2>::type;
    const In* src = reinterpret_cast<const In*>(mc);
    __shared__ double s_x[E * XW];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i = lane & 15, k = lane >> 4;
    const int64_t n_ch = (n_acc + E - 1) / E;
    const int64_t c0 = (int64_t)blockIdx.x * n_ch / gridDim.x;
    const int64_t c1 = (int64_t)(blockIdx.x + 1) * n_ch / gridDim.x;
    const int n_el = E * W;

    // the padding columns 2W .. 16 T stay zero
    for (int e = tid; e < E * XW; e += NT) s_x[e] = 0.0;
    In pre[PRE];
    // element tid + NT q of the chunk (event idx / W, wave idx % W); the
    // address is clamped into the input (n_acc >= 1) and the value
    // multiplied by 0 or 1, so that no load is put behind a branch
    auto load_chunk = [&](int64_t c) {
        const int64_t j0 = c * E;
#pragma unroll
        for (int q = 0; q < PRE; ++q) {
            const int idx = tid + NT * q;
            const int j = idx / W, a = idx - j * W;
            const bool ok = idx < n_el && j0 + j < n_acc;
            const In b = src[ok ? (j0 + j) * W + a : 0];
            const auto keep = ok ? 1.0f : 0.0f;
            pre[q].x = b.x * keep;
            pre[q].y = b.y * keep;
        }
    };
    auto store_chunk = [&]() {
#pragma unroll
        for (int q = 0; q < PRE; ++q) {
            const int idx = tid + NT * q;
            if (idx < n_el) {
                const int j = idx / W, a = idx - j * W;
                s_x[j * XW + a] = (double)pre[q].x;
                s_x[j * XW + W + a] = (double)pre[q].y;
            }
        }
    };
    gd4 d[PPW];
#pragma unroll
    for (int q = 0; q < PPW; ++q) d[q] = gd4{0.0, 0.0, 0.0, 0.0};
    // this wavefront's pairs P0 .. P0 + NP - 1 (pairs t <= u in row-major
    // order) over the staged chunk; every index a constant once unrolled
    auto compute = [&](auto wv) {
        constexpr int P0 = decltype(wv)::value * PPW;
        constexpr int NP = (NPAIR - P0) < PPW ? (NPAIR - P0) : PPW;
        for (int st = 0; st < E / 4; ++st) {
            double x[T];
#pragma unroll
            for (int t = 0; t < T; ++t) x[t] = s_x[(4 * st + k) * XW + 16 * t + i];
            int p = 0;
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int u = t; u < T; ++u, ++p)
                    if (p >= P0 && p < P0 + NP)
                        d[p - P0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t], x[u], d[p - P0],
                                                                         0, 0, 0);
        }
    };
    // 16 wavefronts (more than 8 tiles): the same products with this
    // wavefront's pairs indexed at run time (wavefront-uniform, so scalar),
    // one code path for every wavefront: two LDS reads per pair and step
    // instead of one per tile, within the 128 registers of a 1024-thread block
    int pt[PPW], pu[PPW];
    if constexpr (NW != 4) {
#pragma unroll
        for (int pp = 0; pp < PPW; ++pp) {
            int p = wave * PPW + pp, t = 0;
            if (p >= NPAIR) p = NPAIR - 1;   // past the last pair: never used
            while (p >= T - t) {
                p -= T - t;
                ++t;
            }
            pt[pp] = __builtin_amdgcn_readfirstlane(16 * t);
            pu[pp] = __builtin_amdgcn_readfirstlane(16 * (t + p));
        }
    }
    const int n_mine = NW != 4 ? min(PPW, max(0, NPAIR - wave * PPW)) : 0;
    auto compute_rt = [&]() {
        for (int st = 0; st < E / 4; ++st) {
            const double* row = s_x + (4 * st + k) * XW + i;
#pragma unroll
            for (int pp = 0; pp < PPW; ++pp)
                if (pp < n_mine)
                    d[pp] = __builtin_amdgcn_mfma_f64_16x16x4f64(row[pt[pp]], row[pu[pp]], d[pp],
                                                                 0, 0, 0);
        }
    };
    auto write = [&](auto wv) {
        constexpr int P0 = decltype(wv)::value * PPW;
        constexpr int NP = (NPAIR - P0) < PPW ? (NPAIR - P0) : PPW;
        double* rec = records + (int64_t)blockIdx.x * NPAIR * 256;
#pragma unroll
        for (int pp = 0; pp < NP; ++pp)
#pragma unroll
            for (int r = 0; r < 4; ++r) rec[((P0 + pp) * 4 + r) * 64 + lane] = d[pp][r];
    };
    if (c0 < c1) load_chunk(c0);
    for (int64_t c = c0; c < c1; ++c) {
        __syncthreads();   // the previous chunk's reads (and the zeroing) done
        store_chunk();
        __syncthreads();
        if (c + 1 < c1) load_chunk(c + 1);
        if constexpr (NW == 4) for_wave<NW>(wave, compute, std::make_integer_sequence<int, NW>{});
        else compute_rt();
    }
    if constexpr (NW == 4) {
        for_wave<NW>(wave, write, std::make_integer_sequence<int, NW>{});
    } else {
        double* rec = records + (int64_t)blockIdx.x * NPAIR * 256;
#pragma unroll
        for (int pp = 0; pp < PPW; ++pp)
            if (pp < n_mine)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    rec[((wave * PPW + pp) * 4 + r) * 64 + lane] = d[pp][r];
    }
}

// tiles of 16 components of the MFMA build (0: W too large for it);
// up to 4 tiles k_gram_mfma, 5 to 16 k_gram_mfma_lds
int gram_mfma_tiles(int W)
{
    const int T = (2 * W + 15) / 16;
    return T <= kGramMfmaMaxTiles ? T : 0;
}

// blocks of the matrix-core build: at least 64 steps of 4 events each, up to
// 512 (two wavefronts per SIMD); 256 for the 16-wavefront blocks of more than
// 8 tiles (one block per CU)
int gram_mfma_rows(int64_t n_acc, int W)
{
    int64_t r = ((n_acc + 3) / 4 + 63) / 64;
    const int cap = gram_mfma_tiles(W) > 8 ? kGramMaxRows / 2 : kGramMaxRows;
    if (r > cap) r = cap;
    return (int)(r < 1 ? 1 : r);
}

int gram_mfma_record(int W)
{
    const int T = gram_mfma_tiles(W);
    return T * (T + 1) / 2 * 256;
}

hipError_t launch_gram_mfma(const void* mc, bool c128, int64_t n_acc, int W, double* records,
                            int rows, hipStream_t s, const LaunchEvents& ev)
{
    const int T = gram_mfma_tiles(W);
    const dim3 grid(rows), block(256);
#define PWA_GRAM_MFMA(C, TT)                                                                     \
    hipExtLaunchKernelGGL((k_gram_mfma<C, TT>), grid, block, 0, s, ev.start, ev.stop, 0, mc,  \
                          n_acc, W, records)
#define PWA_GRAM_LDS(C, TT)                                                                      \
    hipExtLaunchKernelGGL((k_gram_mfma_lds<C, TT, gram_lds_waves<TT>()>), grid,               \
                          dim3(64 * gram_lds_waves<TT>()), 0, s, ev.start, ev.stop, 0, mc,    \
                          n_acc, W, records)
    switch (T) {
    case 1: if (c128) PWA_GRAM_MFMA(true, 1); else PWA_GRAM_MFMA(false, 1); break;
    case 2: if (c128) PWA_GRAM_MFMA(true, 2); else PWA_GRAM_MFMA(false, 2); break;
    case 3: if (c128) PWA_GRAM_MFMA(true, 3); else PWA_GRAM_MFMA(false, 3); break;
    case 4: if (c128) PWA_GRAM_MFMA(true, 4); else PWA_GRAM_MFMA(false, 4); break;
    case 5: if (c128) PWA_GRAM_LDS(true, 5); else PWA_GRAM_LDS(false, 5); break;
    case 6: if (c128) PWA_GRAM_LDS(true, 6); else PWA_GRAM_LDS(false, 6); break;
    case 7: if (c128) PWA_GRAM_LDS(true, 7); else PWA_GRAM_LDS(false, 7); break;
    case 8: if (c128) PWA_GRAM_LDS(true, 8); else PWA_GRAM_LDS(false, 8); break;
    case 9: if (c128) PWA_GRAM_LDS(true, 9); else PWA_GRAM_LDS(false, 9); break;
    case 10: if (c128) PWA_GRAM_LDS(true, 10); else PWA_GRAM_LDS(false, 10); break;
    case 11: if (c128) PWA_GRAM_LDS(true, 11); else PWA_GRAM_LDS(false, 11); break;
    case 12: if (c128) PWA_GRAM_LDS(true, 12); else PWA_GRAM_LDS(false, 12); break;
    case 13: if (c128) PWA_GRAM_LDS(true, 13); else PWA_GRAM_LDS(false, 13); break;
    case 14: if (c128) PWA_GRAM_LDS(true, 14); else PWA_GRAM_LDS(false, 14); break;
    case 15: if (c128) PWA_GRAM_LDS(true, 15); else PWA_GRAM_LDS(false, 15); break;
    case 16: if (c128) PWA_GRAM_LDS(true, 16); else PWA_GRAM_LDS(false, 16); break;
    default: return hipErrorInvalidValue;
    }
#undef PWA_GRAM_MFMA
#undef PWA_GRAM_LDS
    return hipGetLastError();
}

// summed Gram tiles -> full Hermitian W x W matrix scaled by 1/N_gen; each
// element of G is read from its upper-triangle copy, so M is Hermitian and its
// diagonal real exactly
__global__ void k_expand_gram(const double* __restrict__ g, int W, int T, double inv_gen,
                              double2* __restrict__ M)
{
    auto G = [&](int r, int c) {
        if (r > c) {
            const int x = r;
            r = c;
            c = x;
        }
        const int t = r >> 4, u = c >> 4;
        const int p = t * T - t * (t - 1) / 2 + (u - t);
        const int row = r & 15, col = c & 15;
        return g[(p * 4 + (row >> 2)) * 64 + (row & 3) * 16 + col];
    };
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < W * W;
         idx += gridDim.x * blockDim.x) {
        const int a = idx / W, b = idx % W;
        const double re = G(a, b) + G(W + a, W + b);
        const double im = G(W + a, b) - G(a, W + b);
        M[idx] = make_double2(re * inv_gen, im * inv_gen);
    }
}

hipError_t launch_expand_gram(const double* colsum, int W, int64_t n_gen, double* M,
                              hipStream_t s)
{
    const int total = W * W;
    hipLaunchKernelGGL(k_expand_gram, dim3((total + 255) / 256), dim3(256), 0, s, colsum, W,
                       gram_mfma_tiles(W), 1.0 / (double)n_gen, (double2*)M);
    return hipGetLastError();
}


// one wavefront per column; lane l sums rows l, l + 64, ... in order.  Rows
// are `stride` doubles apart; the first `cols` columns are summed.
__global__ __launch_bounds__(256) void k_colsum(const double* __restrict__ partials, int rows,
                                                int cols, int stride, double* __restrict__ out)
{
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (col >= cols) return;
    double s = 0.0;
    for (int r = lane; r < rows; r += 64) s += partials[(int64_t)r * stride + col];
    s = wave_allsum(s);
    if (lane == 0) out[col] = s;
}

hipError_t launch_colsum(const double* partials, int rows, int cols, int stride, double* out,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_colsum, dim3((cols + 3) / 4), dim3(256), 0, s, partials, rows, cols,
                       stride, out);
    return hipGetLastError();
}

// ---- end of an evaluation -------------------------------------------------
// Every loop below issues its loads in predicated batches before using any of
// them: a loop that adds each value as it arrives costs one memory round trip
// per element, and the records are few (one per block of the streaming
// kernel), so one or two batches cover a thread's share.
constexpr int kBatch = 16;

// Sum over rows first, first + step, ... (< rows) of the double2 at `col` of
// each record, added in row order.
__device__ inline double2 strided_record_sum(const TailArgs& ta, int col, int first, int step)
{
    double2 acc = make_double2(0.0, 0.0);
    const double* base = ta.rec + col;
    for (int r = first; r < ta.rows; r += kBatch * step) {
        // every load is issued (a row past the last reads the last and is not
        // added), so that none sits behind a branch
        double2 x[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int row = min(r + k * step, ta.rows - 1);
            x[k] = *reinterpret_cast<const double2*>(base + (int64_t)row * ta.rec_len);
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            if (r + k * step < ta.rows) {
                acc.x += x[k].x;
                acc.y += x[k].y;
            }
        }
    }
    return acc;
}

// All of this block's result stores have completed: publish `seq` in its
// completion word (none for the asynchronous entry points: word is null in
// every block).
__device__ inline void publish(unsigned long long* word, unsigned long long seq)
{
    if (!word) return;
    wait_vm_complete();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(word, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// V_a M_ab
__device__ inline double2 v_times_m(const double* v, const double2* M, int W, int a, int b)
{
    const double2 x = M[a * W + b];
    const double vr = v[2 * a], vi = v[2 * a + 1];
    return make_double2(vr * x.x - vi * x.y, vr * x.y + vi * x.x);
}

// Block sums of four values in a fixed order (butterflies in each wavefront,
// then the wavefront sums in wave order), with one LDS round.
__device__ inline double4 block_sum4(double4 x)
{
    __shared__ double4 s_w[kAssembleThreads / 64];
    x.x = wave_allsum(x.x);
    x.y = wave_allsum(x.y);
    x.z = wave_allsum(x.z);
    x.w = wave_allsum(x.w);
    if (lane_id() == 0) s_w[threadIdx.x >> 6] = x;
    __syncthreads();
    double4 r = make_double4(0.0, 0.0, 0.0, 0.0);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        r.x += s_w[w].x;
        r.y += s_w[w].y;
        r.z += s_w[w].z;
        r.w += s_w[w].w;
    }
    return r;
}

// One assembly block over records [sum ln I, n_bad, x_0, ..., x_{W-1}] (x_b
// complex: u_b = sum_a V_a U_ab of the table forms, or g_b of the amplitude
// form; both enter as G_b = 2 (m_b - x_b)).  Role 0 forms the NLL and n_bad,
// role 1 + b the gradient component b.  Every thread issues all of its loads
// (its records in batches of kBatch, its share of M) before adding any, so
// that the whole block waits about one memory round trip per batch; V is
// read from LDS.
__device__ void assemble_role_g(const double* vg, const TailArgs& ta, int role,
                                unsigned long long* word)
{
    __shared__ double s_v[2 * PWA_MAX_WAVES_AMPLITUDE];
    const int W = ta.W;
    for (int e = threadIdx.x; e < 2 * W; e += blockDim.x) s_v[e] = vg[e];
    const double* v = s_v;
    const int NT = blockDim.x;
    const int col = role == 0 ? 0 : 2 * role;   // record column of this role
    const int b = role - 1;
    // M entries of this thread: role 0 all of M (pairs k = a W + b'), role
    // 1 + b column b (k = a); loaded with the first batch of records
    const int n_m = role == 0 ? W * W : W;
    constexpr int kMaxM = 4;
    double2 mv[kMaxM];
#pragma unroll
    for (int q = 0; q < kMaxM; ++q) {
        const int k = threadIdx.x + q * NT;
        mv[q] = k < n_m ? ta.M[role == 0 ? k : k * W + b] : make_double2(0.0, 0.0);
    }
    double2 acc = make_double2(0.0, 0.0);
    const double* base = ta.rec + col;
    for (int r0 = threadIdx.x; r0 < ta.rows; r0 += kBatch * NT) {
        double2 x[kBatch];
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            const int row = r0 + k * NT;
            x[k] = row < ta.rows
                       ? *reinterpret_cast<const double2*>(base + (int64_t)row * ta.rec_len)
                       : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int k = 0; k < kBatch; ++k) {
            acc.x += x[k].x;
            acc.y += x[k].y;
        }
    }
    // the MC term of this thread: role 0 its part of mu = sum Re(conj(V_b') V_a
    // M_ab'); role 1 + b its part of m_b = sum_a V_a M_ab (the rest of M, for
    // W^2 > kMaxM NT, loaded here)
    double2 mt = make_double2(0.0, 0.0);
    auto add_m = [&](int k, double2 x) {
        const int a = role == 0 ? k / W : k;
        const double vr = v[2 * a], vi = v[2 * a + 1];
        const double tr = vr * x.x - vi * x.y, ti = vr * x.y + vi * x.x;   // V_a M_ab'
        if (role == 0) {
            const int bb = k % W;
            mt.x += v[2 * bb] * tr + v[2 * bb + 1] * ti;
        } else {
            mt.x += tr;
            mt.y += ti;
        }
    };
    __syncthreads();   // s_v
#pragma unroll
    for (int q = 0; q < kMaxM; ++q)
        if (threadIdx.x + q * NT < n_m) add_m(threadIdx.x + q * NT, mv[q]);
    // the rest of M (W^2 > kMaxM NT), in the same order, kMaxM loads at a
    // time issued before any is used (an entry past the last reads the last
    // and is not added)
    for (int k0 = threadIdx.x + kMaxM * NT; k0 < n_m; k0 += kMaxM * NT) {
        double2 xm[kMaxM];
#pragma unroll
        for (int q = 0; q < kMaxM; ++q) {
            const int k = min(k0 + q * NT, n_m - 1);
            xm[q] = ta.M[role == 0 ? k : k * W + b];
        }
#pragma unroll
        for (int q = 0; q < kMaxM; ++q)
            if (k0 + q * NT < n_m) add_m(k0 + q * NT, xm[q]);
    }
    const double4 tot = block_sum4(make_double4(acc.x, acc.y, mt.x, mt.y));
    if (threadIdx.x == 0) {
        if (role == 0) {
            // tot.x = sum ln I, tot.y = n_bad, tot.z = mu
            store_system(ta.out, tot.y > 0.0 ? INFINITY : (-tot.x + tot.z));
            store_system(ta.out + 1, tot.y);
        } else {
            // a degenerate event made its records' entries NaN, and so G_b
            store_system(ta.out + 2 + 2 * b, 2.0 * (tot.z - tot.x));
            store_system(ta.out + 3 + 2 * b, 2.0 * (tot.w - tot.y));
        }
    }
    publish(word, ta.seq);
}

// One assembly block over packed-U records [sum ln I, n_bad, U_e (2P)] (the
// plain FP64 form): role 0 forms the NLL, role 1 + b the gradient component b
// from the W packed entries of its row and column; V (2W doubles) at v; ends
// by publishing in `word`.
__device__ void assemble_role(const double* v, const TailArgs& ta, int role,
                              unsigned long long* word)
{
    if (ta.g_records) {
        assemble_role_g(v, ta, role, word);
        return;
    }
    __shared__ double s_wave[kAssembleThreads / 64];
    __shared__ double2 s_acc[kAssembleThreads];
    const int W = ta.W;
    if (role == 0) {
        // columns 0 and 1: sum ln I and the count of invalid intensities
        const double2 head = strided_record_sum(ta, 0, threadIdx.x, blockDim.x);
        const double dsum = block_sum_fixed(head.x, s_wave);
        const double nbad = block_sum_fixed(head.y, s_wave);
        // mu = sum_{a,b} Re(conj(V_b) V_a M_ab): pairs (a, b) over the threads
        double mu_part = 0.0;
        for (int k = threadIdx.x; k < W * W; k += blockDim.x) {
            const int a = k / W, bb = k % W;
            const double2 t = v_times_m(v, ta.M, W, a, bb);
            mu_part += v[2 * bb] * t.x + v[2 * bb + 1] * t.y;
        }
        const double mu = block_sum_fixed(mu_part, s_wave);
        if (threadIdx.x == 0) {
            store_system(ta.out, nbad > 0.0 ? INFINITY : (-dsum + mu));
            store_system(ta.out + 1, nbad);
        }
        publish(word, ta.seq);
        return;
    }
    const int b = role - 1;
    // the entries this gradient component needs: U_ab for all a (packed row and
    // column of b); thread t works on entry a = t % W over the record range
    // t / W, and the ranges are added in order
    const int nent = W;
    const int chunks = kAssembleThreads / nent;
    const int a = threadIdx.x % nent;
    const int ch = threadIdx.x / nent;
    double2 acc = make_double2(0.0, 0.0);
    if (ch < chunks) {
        int col;
        double sgn = 1.0;
        if (a <= b) {
            col = 2 + 2 * packed_index(W, a, b);
        } else {
            col = 2 + 2 * packed_index(W, b, a);   // U_ab = conj(U_ba)
            sgn = -1.0;
        }
        acc = strided_record_sum(ta, col, ch, chunks);
        acc.y *= sgn;
    }
    s_acc[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < 64) {
        // lane l: u term of entry l (its chunk partials in chunk order) and the
        // MC terms V_a M_ab of a = l, l + 64, ...; then fixed butterflies
        const int l = threadIdx.x;
        double ur = 0.0, ui = 0.0, mr = 0.0, mi = 0.0;
        if (l < nent) {
            double xr = 0.0, xi = 0.0;
            for (int c = 0; c < chunks; ++c) {
                xr += s_acc[c * nent + l].x;
                xi += s_acc[c * nent + l].y;
            }
            const double vr = v[2 * l], vi = v[2 * l + 1];
            ur = vr * xr - vi * xi;
            ui = vr * xi + vi * xr;
        }
        for (int aa = l; aa < W; aa += 64) {
            const double2 t = v_times_m(v, ta.M, W, aa, b);
            mr += t.x;
            mi += t.y;
        }
        ur = wave_allsum(ur);
        ui = wave_allsum(ui);
        mr = wave_allsum(mr);
        mi = wave_allsum(mi);
        if (l == 0) {
            const double gr = 2.0 * (mr - ur), gi = 2.0 * (mi - ui);
            // a degenerate event made its records' entries NaN, and so G_b
            store_system(ta.out + 2 + 2 * b, gr);
            store_system(ta.out + 3 + 2 * b, gi);
        }
    }
    publish(word, ta.seq);
}

__global__ __launch_bounds__(kAssembleThreads) void k_assemble(VParams vp, TailArgs ta)
{
    assemble_role(vsrc(vp), ta, blockIdx.x, ta.done ? ta.done + blockIdx.x : nullptr);
}

// The assembly of many evaluations in one launch: block i is role
// blocks[i].role of job blocks[i].job.  The completion value is read from the
// head of the parameter buffer, so that a captured graph can replay the launch
// with new parameters and a new value.
__global__ __launch_bounds__(kAssembleThreads) void k_assemble_multi(
    const MultiJob* __restrict__ jobs, const AsmBlock* __restrict__ blocks,
    const double* __restrict__ params, const double* __restrict__ recs, int rec_stride,
    double* out, unsigned long long* done)
{
    const AsmBlock ab = blocks[blockIdx.x];
    const MultiJob j = jobs[ab.job];
    TailArgs ta;
    ta.rec = recs + (int64_t)j.rec0 * rec_stride;
    ta.rows = j.nrec;
    ta.rec_len = rec_stride;
    ta.M = j.M;
    ta.out = out + j.out_off;
    ta.done = done;
    ta.seq = *reinterpret_cast<const unsigned long long*>(params);
    ta.W = j.W;
    ta.grad = 1;
    ta.g_records = 1;
    assemble_role(params + j.v_off, ta, ab.role, done + j.done_off + ab.role);
}

hipError_t launch_assemble_multi(const MultiLaunch& ml, hipStream_t s)
{
    hipLaunchKernelGGL(k_assemble_multi, dim3(ml.n_asm), dim3(kAssembleThreads), 0, s, ml.jobs,
                       ml.asm_blocks, ml.params, ml.recs, ml.rec_stride, ml.out, ml.done);
    return hipGetLastError();
}

int assemble_blocks(int W, bool grad) { return 1 + (grad ? W : 0); }

hipError_t launch_assemble(const VParams& vp, const TailArgs& ta, hipStream_t s)
{
    hipLaunchKernelGGL(k_assemble, dim3(assemble_blocks(ta.W, ta.grad != 0)),
                       dim3(kAssembleThreads), 0, s, vp, ta);
    return hipGetLastError();
}

}  // namespace pwa
