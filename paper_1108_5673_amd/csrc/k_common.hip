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

// NLL and gradient from the column sums, by the block that finishes last.
//
// Every block of k_reduce_finalize sums four columns of the partial records
// (one wavefront per column, as k_colsum).  It then takes a ticket; the block
// that draws the last ticket knows all column sums are written and assembles
//   mu   = sum_b Re(conj(V_b) m_b),  m_b = sum_a V_a M_ab
//   NLL  = -sum ln I + mu
//   G_b  = 2 (m_b - u_b),  u_b = sum_a V_a U_ab   (table forms, U Hermitian packed)
//   G_b  = 2 (m_b - g_b)                          (amplitude form)
// with thread t working on wave b = t % W and the a-range t / W, partial sums
// combined in LDS in a fixed order.  The result goes straight to `out`, a
// pinned host buffer, and the ticket counter is reset for the next call.
constexpr int kFinBlock = 256;

__device__ inline void finalize_block(const double* __restrict__ colsum,
                                      const double2* __restrict__ M, int W, const VParams& vp,
                                      bool grad, bool amplitude, double* __restrict__ out)
{
    __shared__ double s_part[4][kFinBlock];
    __shared__ double s_mu[kFinBlock];
    const int t = threadIdx.x;
    const int groups = W <= kFinBlock ? kFinBlock / W : 1;   // a-ranges per wave
    const int b = t % W;
    const int g = t / W;
    double mr = 0.0, mi = 0.0, ur = 0.0, ui = 0.0;
    if (g < groups) {
        for (int a = g; a < W; a += groups) {
            const double vr = vp.v[2 * a], vi = vp.v[2 * a + 1];
            const double2 x = M[a * W + b];
            mr += vr * x.x - vi * x.y;
            mi += vr * x.y + vi * x.x;
            if (grad && !amplitude) {
                double xr, xi;
                if (a <= b) {
                    const int e = packed_index(W, a, b);
                    xr = colsum[2 + 2 * e];
                    xi = colsum[3 + 2 * e];
                } else {
                    const int e = packed_index(W, b, a);
                    xr = colsum[2 + 2 * e];
                    xi = -colsum[3 + 2 * e];
                }
                ur += vr * xr - vi * xi;
                ui += vr * xi + vi * xr;
            }
        }
    }
    s_part[0][t] = mr;
    s_part[1][t] = mi;
    s_part[2][t] = ur;
    s_part[3][t] = ui;
    __syncthreads();
    const double nbad = colsum[1];
    if (t < W) {
        double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
        for (int gg = 0; gg < groups; ++gg) {
            const int src = gg * W + t;
            r0 += s_part[0][src];
            r1 += s_part[1][src];
            r2 += s_part[2][src];
            r3 += s_part[3][src];
        }
        s_mu[t] = vp.v[2 * t] * r0 + vp.v[2 * t + 1] * r1;
        if (grad) {
            double gr, gi;
            if (amplitude) {
                gr = 2.0 * (r0 - colsum[2 + 2 * t]);
                gi = 2.0 * (r1 - colsum[3 + 2 * t]);
            } else {
                gr = 2.0 * (r0 - r2);
                gi = 2.0 * (r1 - r3);
            }
            out[2 + 2 * t] = nbad > 0.0 ? NAN : gr;
            out[3 + 2 * t] = nbad > 0.0 ? NAN : gi;
        }
    }
    __syncthreads();
    if (t == 0) {
        double mu = 0.0;
        for (int bb = 0; bb < W; ++bb) mu += s_mu[bb];
        out[0] = nbad > 0.0 ? INFINITY : (-colsum[0] + mu);
        out[1] = nbad;
    }
}

__global__ __launch_bounds__(kFinBlock) void k_reduce_finalize(
    const double* __restrict__ partials, int rows, int cols, int stride, double* __restrict__ colsum,
    unsigned int* __restrict__ ticket, const double2* __restrict__ M, int W, VParams vp, bool grad,
    bool amplitude, double* __restrict__ out)
{
    __shared__ bool s_last;
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (col < cols) {
        double s = 0.0;
        for (int r = lane; r < rows; r += 64) s += partials[(int64_t)r * stride + col];
        s = wave_allsum(s);
        if (lane == 0) colsum[col] = s;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    finalize_block(colsum, M, W, vp, grad, amplitude, out);
    if (threadIdx.x == 0) atomicExch(ticket, 0u);
}

hipError_t launch_reduce_finalize(const Model& m, const VParams& vp, bool grad, double* out,
                                  hipStream_t s)
{
    const int cols = grad ? m.rec_len : 2;
    hipLaunchKernelGGL(k_reduce_finalize, dim3((cols + 3) / 4), dim3(kFinBlock), 0, s,
                       m.d_partials, m.rows, cols, m.rec_len, m.d_colsum, m.d_ticket,
                       (const double2*)m.d_M, m.W, vp, grad, m.form == kAmp32, out);
    return hipGetLastError();
}

}  // namespace pwa
