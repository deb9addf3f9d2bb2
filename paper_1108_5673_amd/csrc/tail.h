// tail.h -- the end of every evaluation: the fixed-order sums over the
// streaming kernel's per-block partial records and the assembly of the NLL and
// its gradient, in one small kernel launched after the streaming kernel.
//
// Record layout (rec_len doubles): [sum ln I, n_bad, then 2 doubles per
// accumulated entry: U_e of the packed table (table forms, e < P), or g_b =
// sum_i S_i conj(A_ib) / I_i (amplitude form, b < W)].
//
// The kernel boundary makes every block's record visible with ordinary stores
// and loads; no kernel synchronises across blocks.  (Cross-block tickets at
// the end of a persistent streaming kernel proved costly on this part: a
// device-scope fence writes back and invalidates the issuing XCD's whole L2,
// and contended device-scope atomics serialise.)
//
// The assembly is split by output so that its blocks are independent:
//   block 0      NLL = -sum ln I + mu,  mu = sum_b Re(conj(V_b) m_b),
//                m_b = sum_a V_a M_ab (the MC term of Eq. 3), and n_bad;
//   block 1 + b  G_b = 2 (m_b - u_b),  u_b = sum_a V_a U_ab  (packed U records;
//                U is Hermitian and stored packed, so block b reads only the
//                W packed columns of its row and column), or
//                G_b = 2 (m_b - g_b)  (g records).
// A degenerate event (I <= 0 or not finite) is counted in n_bad, which makes
// the NLL +inf, and carries a NaN weight, which makes every U_ab or g_b of its
// block's record, and so every G_b, NaN.
// Every sum over records runs in a fixed order.  Each block writes its outputs
// to pinned host memory with system-scope stores, waits for their completion
// and then stores `seq` in its own completion word; the host waits for all of
// them.
#pragma once

#include <hip/hip_runtime.h>

#include "pwa_internal.h"
#include "wave_ops.h"

namespace pwa {

struct TailArgs {
    const double* rec;       // rows x rec_len partial records
    int rows;
    int rec_len;             // doubles per record
    const double2* M;        // W x W MC matrix
    double* out;             // [nll, n_bad, grad 2W] (pinned host memory)
    unsigned long long* done;   // one completion word per assembly block (pinned host memory)
    unsigned long long seq;     // value published in the completion words
    int W;
    int grad;
    int g_records;           // records hold g_b (2W) rather than packed U (2P)
};

constexpr int kAssembleThreads = 256;

__device__ inline void store_system(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Block sum in a fixed order: a butterfly inside each wavefront, then the
// wavefront sums in wave order (blockDim a multiple of 64, at most 1024).
__device__ inline double block_sum_fixed(double x, double* s_wave)
{
    x = wave_allsum(x);
    const int waves = blockDim.x >> 6;
    if (lane_id() == 0) s_wave[threadIdx.x >> 6] = x;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < waves; ++w) r += s_wave[w];
    __syncthreads();
    return r;
}

// Wait until this thread's outstanding vector-memory operations completed.
__device__ inline void wait_vm_complete()
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

}  // namespace pwa
