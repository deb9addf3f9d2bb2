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

// NLL and gradient from the column sums; one block, thread b handles wave b.
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ colsum,
                                                  const double2* __restrict__ M, int W,
                                                  int rec_len, VParams vp, bool grad,
                                                  bool amplitude, double* __restrict__ out)
{
    __shared__ double s_mu[PWA_MAX_WAVES_AMPLITUDE];
    const double sum_ln = colsum[0];
    const double nbad = colsum[1];
    for (int b = threadIdx.x; b < W; b += blockDim.x) {
        // m_b = sum_a V_a M_ab
        double mr = 0.0, mi = 0.0;
        for (int a = 0; a < W; ++a) {
            const double vr = vp.v[2 * a], vi = vp.v[2 * a + 1];
            const double2 x = M[a * W + b];
            mr += vr * x.x - vi * x.y;
            mi += vr * x.y + vi * x.x;
        }
        // Re( conj(V_b) m_b )
        s_mu[b] = vp.v[2 * b] * mr + vp.v[2 * b + 1] * mi;
        if (grad) {
            double gr, gi;
            if (amplitude) {
                gr = 2.0 * (mr - colsum[2 + 2 * b]);
                gi = 2.0 * (mi - colsum[3 + 2 * b]);
            } else {
                // u_b = sum_a V_a U_ab, U Hermitian, stored packed (a <= b)
                double ur = 0.0, ui = 0.0;
                for (int a = 0; a < W; ++a) {
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
                    const double vr = vp.v[2 * a], vi = vp.v[2 * a + 1];
                    ur += vr * xr - vi * xi;
                    ui += vr * xi + vi * xr;
                }
                gr = 2.0 * (mr - ur);
                gi = 2.0 * (mi - ui);
            }
            out[2 + 2 * b] = nbad > 0.0 ? NAN : gr;
            out[3 + 2 * b] = nbad > 0.0 ? NAN : gi;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double mu = 0.0;
        for (int b = 0; b < W; ++b) mu += s_mu[b];
        out[0] = nbad > 0.0 ? INFINITY : (-sum_ln + mu);
        out[1] = nbad;
    }
    (void)rec_len;
}

hipError_t launch_finalize(const Model& m, const VParams& vp, bool grad, double* out,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, m.d_colsum,
                       (const double2*)m.d_M, m.W, m.rec_len, vp, grad, m.form == kAmp32, out);
    return hipGetLastError();
}

}  // namespace pwa
