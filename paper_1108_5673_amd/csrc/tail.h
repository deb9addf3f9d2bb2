// tail.h -- the end of every evaluation: the fixed-order sum of the streaming
// kernel's per-block partial records and the assembly of the NLL and its
// gradient, in one small kernel launched after the streaming kernel (the
// kernel boundary makes every block's record visible; a device-wide fence per
// streaming block would cost a full L2 write-back and invalidate each).
//
// Record layout (rec_len doubles): [sum ln I, n_bad, then 2 doubles per
// accumulated entry: U_e (table forms, e < P) or g_b (amplitude form, b < W)].
//
// Each block of k_reduce_assemble sums 64 columns over all records (16 row
// groups of 64 lanes, four interleaved accumulators per lane, then the 16
// groups in order), takes a ticket, and the block that draws the last one
// assembles
//   mu  = sum_b Re(conj(V_b) m_b),  m_b = sum_a V_a M_ab       (MC term, Eq. 3)
//   NLL = -sum ln I + mu
//   G_b = 2 (m_b - u_b),  u_b = sum_a V_a U_ab   (table forms, U Hermitian packed)
//   G_b = 2 (m_b - g_b)                          (amplitude form)
// into `out` (pinned host memory), then publishes `seq` in `done` so the host
// can stop waiting.  The ticket is reset by the block that consumed it.
#pragma once

#include <hip/hip_runtime.h>

#include "pwa_internal.h"
#include "wave_ops.h"

namespace pwa {

constexpr int kReduceThreads = 1024;   // 16 row groups x 64 columns
constexpr int kReduceCols = 64;

struct TailArgs {
    const double* partials;  // rows x rec_len block records
    int rows;
    double* colsum;          // rec_len final sums
    unsigned int* ticket;    // last-block counter, zero between calls
    const double2* M;        // W x W MC matrix
    double* out;             // [nll, n_bad, grad 2W] (pinned host memory)
    unsigned long long* done;   // completion word (pinned host memory)
    unsigned long long seq;     // value published in *done at the end
    int rec_len;             // doubles per record
    int cols;                // leading columns that carry data (2 without gradient)
    int W;
    int grad;
    int amplitude;
};

// LDS scratch the assembly needs, in doubles, for a block of `threads` threads.
__host__ __device__ constexpr int tail_scratch_doubles(int threads)
{
    return 4 * (threads < 256 ? threads : 256) + PWA_MAX_WAVES_AMPLITUDE;
}

__device__ inline void tail_assemble(const TailArgs& ta, const VParams& vp, double* scratch)
{
    const int nthr = blockDim.x < 256 ? blockDim.x : 256;
    double* s_part[4] = {scratch, scratch + nthr, scratch + 2 * nthr, scratch + 3 * nthr};
    double* s_mu = scratch + 4 * nthr;
    const double* colsum = ta.colsum;
    const int W = ta.W;
    const int t = threadIdx.x;
    // thread t < nthr works on wave b = t % W over the a-range t / W
    const int groups = (W <= nthr) ? nthr / W : 1;
    double mr = 0.0, mi = 0.0, ur = 0.0, ui = 0.0;
    if (t < nthr) {
        const int b = t % W;
        const int g = t / W;
        if (g < groups) {
            for (int a = g; a < W; a += groups) {
                const double vr = vp.v[2 * a], vi = vp.v[2 * a + 1];
                const double2 x = ta.M[a * W + b];
                mr += vr * x.x - vi * x.y;
                mi += vr * x.y + vi * x.x;
                if (ta.grad && !ta.amplitude) {
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
    }
    __syncthreads();
    const double nbad = colsum[1];
    for (int b = t; b < W; b += blockDim.x) {
        double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;
        if (W <= nthr) {
            for (int gg = 0; gg < groups; ++gg) {
                const int src = gg * W + b;
                r0 += s_part[0][src];
                r1 += s_part[1][src];
                r2 += s_part[2][src];
                r3 += s_part[3][src];
            }
        } else {
            // more waves than threads (W > blockDim): direct sums
            for (int a = 0; a < W; ++a) {
                const double vr = vp.v[2 * a], vi = vp.v[2 * a + 1];
                const double2 x = ta.M[a * W + b];
                r0 += vr * x.x - vi * x.y;
                r1 += vr * x.y + vi * x.x;
            }
        }
        s_mu[b] = vp.v[2 * b] * r0 + vp.v[2 * b + 1] * r1;
        if (ta.grad) {
            double gr, gi;
            if (ta.amplitude) {
                gr = 2.0 * (r0 - colsum[2 + 2 * b]);
                gi = 2.0 * (r1 - colsum[3 + 2 * b]);
            } else {
                gr = 2.0 * (r0 - r2);
                gi = 2.0 * (r1 - r3);
            }
            ta.out[2 + 2 * b] = nbad > 0.0 ? NAN : gr;
            ta.out[3 + 2 * b] = nbad > 0.0 ? NAN : gi;
        }
    }
    __syncthreads();
    if (t == 0) {
        double mu = 0.0;
        for (int b = 0; b < W; ++b) mu += s_mu[b];
        ta.out[0] = nbad > 0.0 ? INFINITY : (-colsum[0] + mu);
        ta.out[1] = nbad;
        __threadfence_system();
        __hip_atomic_store(ta.done, ta.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace pwa
