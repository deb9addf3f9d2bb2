// k_common.hip -- the MC integral matrix and the fixed-order final reduction.
//
// M_aa' = (1/N_gen) sum_{j accepted} B_ja B*_ja' (Eq. 3, inner bracket) is built
// once per model in FP64.  Each evaluation ends with two small kernels: a
// column sum of the per-block partial records (one wavefront per column, a
// fixed assignment of rows to lanes and a fixed butterfly, so results repeat
// bit for bit), then the assembly of NLL = -sum ln I + mu and
// G_b = 2 sum_a V_a (M_ab - U_ab) (table forms) or 2 sum_a V_a M_ab - 2 g_b
// (amplitude form), with mu = sum_a sum_b V_a V*_b M_ab: the MC quadratic form
// is evaluated here, in FP64, once per evaluation.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pwa_internal.h"
#include "tail.h"
#include "wave_ops.h"

namespace pwa {

constexpr int kGramChunk = 32;     // MC events staged in LDS at a time
constexpr int kGramMaxRows = 512;  // partial records of the MC matrix build
constexpr int kGramMaxSlots = 33;  // entries per thread: P <= 256 * 33 (W <= 128)

int gram_rows(int64_t n_acc)
{
    int64_t chunks = (n_acc + kGramChunk - 1) / kGramChunk;
    if (chunks > kGramMaxRows) chunks = kGramMaxRows;
    return (int)(chunks < 1 ? 1 : chunks);
}

template <bool C128>
__global__ __launch_bounds__(256) void k_gram(const void* __restrict__ mc, int64_t n_acc, int W,
                                              int P, const uint32_t* __restrict__ pairs,
                                              double* __restrict__ partials)
{
    extern __shared__ double2 s_b[];   // kGramChunk x W
    const int64_t nch = (n_acc + kGramChunk - 1) / kGramChunk;
    const int64_t c0 = (int64_t)blockIdx.x * nch / gridDim.x;
    const int64_t c1 = (int64_t)(blockIdx.x + 1) * nch / gridDim.x;
    double ar[kGramMaxSlots], ai[kGramMaxSlots];
    int pa[kGramMaxSlots], pb[kGramMaxSlots];
#pragma unroll
    for (int r = 0; r < kGramMaxSlots; ++r) {
        ar[r] = 0.0;
        ai[r] = 0.0;
        const int e = threadIdx.x + 256 * r;
        const uint32_t pr = (e < P) ? pairs[e] : 0u;
        pa[r] = (int)(pr & 0xffffu);
        pb[r] = (int)(pr >> 16);
    }

    for (int64_t c = c0; c < c1; ++c) {
        for (int idx = threadIdx.x; idx < kGramChunk * W; idx += blockDim.x) {
            const int64_t j = c * kGramChunk + idx / W;
            const int a = idx % W;
            double2 x = make_double2(0.0, 0.0);
            if (j < n_acc) {
                if (C128) x = reinterpret_cast<const double2*>(mc)[j * W + a];
                else {
                    const float2 f = reinterpret_cast<const float2*>(mc)[j * W + a];
                    x = make_double2(f.x, f.y);
                }
            }
            s_b[idx] = x;
        }
        __syncthreads();
        for (int j = 0; j < kGramChunk; ++j) {
#pragma unroll
            for (int r = 0; r < kGramMaxSlots; ++r) {
                if (threadIdx.x + 256 * r < P) {
                    const double2 x = s_b[j * W + pa[r]], y = s_b[j * W + pb[r]];
                    ar[r] += x.x * y.x + x.y * y.y;    // Re x conj(y)
                    ai[r] += x.y * y.x - x.x * y.y;    // Im x conj(y)
                }
            }
        }
        __syncthreads();
    }
    double* rec = partials + (int64_t)blockIdx.x * 2 * P;
#pragma unroll
    for (int r = 0; r < kGramMaxSlots; ++r) {
        const int e = threadIdx.x + 256 * r;
        if (e < P) {
            rec[2 * e] = ar[r];
            rec[2 * e + 1] = ai[r];
        }
    }
}

hipError_t launch_gram(const void* mc, bool c128, int64_t n_acc, int W, int P,
                       const uint32_t* pairs, double* partials, int rows, hipStream_t s)
{
    const size_t lds = sizeof(double2) * kGramChunk * W;
    if (c128)
        hipLaunchKernelGGL(k_gram<true>, dim3(rows), dim3(256), lds, s, mc, n_acc, W, P, pairs,
                           partials);
    else
        hipLaunchKernelGGL(k_gram<false>, dim3(rows), dim3(256), lds, s, mc, n_acc, W, P, pairs,
                           partials);
    return hipGetLastError();
}

// packed column sums (2P doubles) -> full Hermitian W x W matrix scaled by 1/N_gen
__global__ void k_expand_m(const double* __restrict__ packed, int W, double inv_gen,
                           double2* __restrict__ M)
{
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < W * W;
         idx += gridDim.x * blockDim.x) {
        const int a = idx / W, b = idx % W;
        double2 x;
        if (a <= b) {
            const int e = packed_index(W, a, b);
            x = make_double2(packed[2 * e] * inv_gen, packed[2 * e + 1] * inv_gen);
        } else {
            const int e = packed_index(W, b, a);
            x = make_double2(packed[2 * e] * inv_gen, -packed[2 * e + 1] * inv_gen);
        }
        if (a == b) x.y = 0.0;
        M[idx] = x;
    }
}

hipError_t launch_expand_m(const double* packed_colsum, int W, int64_t n_gen, double* M,
                           hipStream_t s)
{
    const int total = W * W;
    hipLaunchKernelGGL(k_expand_m, dim3((total + 255) / 256), dim3(256), 0, s, packed_colsum, W,
                       1.0 / (double)n_gen, (double2*)M);
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

__global__ __launch_bounds__(kReduceThreads) void k_reduce_assemble(VParams vp, TailArgs ta)
{
    __shared__ double s_sum[16][kReduceCols];
    __shared__ double s_scratch[tail_scratch_doubles(kReduceThreads)];
    __shared__ bool s_last;
    const int l = threadIdx.x & 63;
    const int g = threadIdx.x >> 6;                 // row group 0..15
    const int col = blockIdx.x * kReduceCols + l;
    const int64_t stride = ta.rec_len;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (col < ta.cols) {
        int r = g;
        for (; r + 48 < ta.rows; r += 64) {
            s0 += ta.partials[(int64_t)r * stride + col];
            s1 += ta.partials[(int64_t)(r + 16) * stride + col];
            s2 += ta.partials[(int64_t)(r + 32) * stride + col];
            s3 += ta.partials[(int64_t)(r + 48) * stride + col];
        }
        for (; r < ta.rows; r += 16) s0 += ta.partials[(int64_t)r * stride + col];
    }
    s_sum[g][l] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (g == 0 && col < ta.cols) {
        double s = 0.0;
        for (int k = 0; k < 16; ++k) s += s_sum[k][l];
        ta.colsum[col] = s;
    }
    if (gridDim.x > 1) {
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) s_last = atomicAdd(ta.ticket, 1u) == gridDim.x - 1;
        __syncthreads();
        if (!s_last) return;
        __threadfence();
    } else {
        __syncthreads();
    }
    tail_assemble(ta, vp, s_scratch);
    if (threadIdx.x == 0 && gridDim.x > 1) atomicExch(ta.ticket, 0u);
}

hipError_t launch_reduce_assemble(const VParams& vp, const TailArgs& ta, hipStream_t s)
{
    const int blocks = (ta.cols + kReduceCols - 1) / kReduceCols;
    hipLaunchKernelGGL(k_reduce_assemble, dim3(blocks), dim3(kReduceThreads), 0, s, vp, ta);
    return hipGetLastError();
}

}  // namespace pwa
