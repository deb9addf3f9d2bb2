// k_amp.hip -- amplitude-form NLL + gradient (Eq. 1 inside Eq. 3): the
// per-event work is S_i = sum_a V_a A_ia and I_i = |S_i|^2, so only N x W
// amplitudes are streamed instead of the N x W(W+1)/2 table.
//
// Layout (lane-split).  An event is held by q = 2^lq neighbouring lanes, each
// with wl (even) of its waves, so rows are q wl >= W waves long (the extra
// waves are zero; shape per W in amp_shape).  The events form steps of
// R = 64 / q: in step k, lane l takes event k R + (l >> lq) and the waves
// (l & (q - 1)) wl ... + wl - 1 as wl / 2 vectors of two complex64, stored
// [k][vector][lane], so that every load of a wavefront reads 1 KB contiguous.
// Events are padded with zero rows to a multiple of 64.
//
// A wavefront streams a contiguous range of steps through registers
// (non-temporal loads into two register buffers: the next step is in flight
// while the current one is processed):
//   1. S over the lane's waves in FP64, summed over the q lanes of the event
//      by an xor butterfly (every lane of the event ends with the same bits);
//   2. I = |S|^2; in each run of q steps one lane of every event keeps I, so
//      that one logarithm per lane covers the 64 events of the run;
//   3. c = S / I (reciprocal refined in FP64), and per lane, in FP64 registers,
//      g_a += c conj(A_a) over its own waves.
// At the end the lanes that share waves are summed through LDS in lane order,
// the block's wavefronts in wavefront order, and the block writes one record
// [sum ln I, n_bad, g_0, ..., g_{W-1}]; G_b = 2 sum_a V_a M_ab - 2 g_b.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pwa_internal.h"
#include "tail.h"
#include "wave_ops.h"

namespace pwa {

constexpr int kAmpBlockWaves = 4;

template <int WL>
struct AmpRegs {
    float4 x[WL / 2];
};

// The lane's vectors of one step; p points at the step's first vector + lane.
template <int WL>
__device__ inline void amp_load(AmpRegs<WL>& r, const float4* __restrict__ p)
{
    typedef float f4v __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int j = 0; j < WL / 2; ++j) {
        const f4v t = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p + j * 64));
        r.x[j] = make_float4(t.x, t.y, t.z, t.w);
    }
}

// Sum over the 2^lq lanes of an event (xor butterfly; lq is wave-uniform).
__device__ inline double event_lanes_sum(double x, int lq)
{
    if (lq > 0) x += xor_lane_f64<1>(x);
    if (lq > 1) x += xor_lane_f64<2>(x);
    if (lq > 2) x += xor_lane_f64<4>(x);
    if (lq > 3) x += xor_lane_f64<8>(x);
    return x;
}

template <int WL>
struct AmpLane {
    const double2* v;        // V of this lane's waves (LDS)
    double gr[WL], gi[WL];   // sum over its events of c conj(A_a)
    double dsum;             // ln I of the events whose logarithm it has taken
    double held;             // intensity waiting for its logarithm (1 when none)
    int nbad;                // invalid intensities (counted by one lane per event)
};

template <int WL, bool GRAD>
__device__ inline void amp_step(AmpRegs<WL>& r, AmpLane<WL>& st, int64_t evt, int64_t n_events,
                                int lq, int sub, int u)
{
    // V is read from LDS at every step rather than held in registers
    asm volatile("" ::: "memory");
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int j = 0; j < WL / 2; ++j) {
        const float4 x = r.x[j];
        const double2 v0 = st.v[2 * j], v1 = st.v[2 * j + 1];
        sr = __fma_rn(v0.x, (double)x.x, sr);
        sr = __fma_rn(-v0.y, (double)x.y, sr);
        si = __fma_rn(v0.x, (double)x.y, si);
        si = __fma_rn(v0.y, (double)x.x, si);
        sr = __fma_rn(v1.x, (double)x.z, sr);
        sr = __fma_rn(-v1.y, (double)x.w, sr);
        si = __fma_rn(v1.x, (double)x.w, si);
        si = __fma_rn(v1.y, (double)x.z, si);
    }
    if (GRAD) {
        // convert again for step 3 instead of keeping FP64 copies alive
#pragma unroll
        for (int j = 0; j < WL / 2; ++j)
            asm volatile("" : "+v"(r.x[j].x), "+v"(r.x[j].y), "+v"(r.x[j].z), "+v"(r.x[j].w));
    }
    sr = event_lanes_sum(sr, lq);
    si = event_lanes_sum(si, lq);
    const double I = sr * sr + si * si;
    const bool valid = evt < n_events;
    const bool ok = valid && (I > 0.0) && (I < INFINITY);
    if (sub == 0 && valid && !ok) ++st.nbad;
    if (sub == u && ok) st.held = I;
    if (u == (1 << lq) - 1) {
        st.dsum += log(st.held);
        st.held = 1.0;
    }
    if (GRAD) {
        // NaN for a degenerate event (the gradient becomes NaN), 0 for padding
        const double w = ok ? recip_f64(I) : (valid ? NAN : 0.0);
        const double cr = sr * w, ci = si * w;
#pragma unroll
        for (int j = 0; j < WL / 2; ++j) {
            const float4 x = r.x[j];
            st.gr[2 * j] = __fma_rn(cr, (double)x.x, st.gr[2 * j]);
            st.gr[2 * j] = __fma_rn(ci, (double)x.y, st.gr[2 * j]);
            st.gi[2 * j] = __fma_rn(ci, (double)x.x, st.gi[2 * j]);
            st.gi[2 * j] = __fma_rn(-cr, (double)x.y, st.gi[2 * j]);
            st.gr[2 * j + 1] = __fma_rn(cr, (double)x.z, st.gr[2 * j + 1]);
            st.gr[2 * j + 1] = __fma_rn(ci, (double)x.w, st.gr[2 * j + 1]);
            st.gi[2 * j + 1] = __fma_rn(ci, (double)x.z, st.gi[2 * j + 1]);
            st.gi[2 * j + 1] = __fma_rn(-cr, (double)x.w, st.gi[2 * j + 1]);
        }
    }
}

// One block's share of one evaluation: steps [k0, k1) of the amplitudes at
// `amp` (shape lq, WL), V (2W doubles) at `v`; one record to `rec`.
template <int WL, bool GRAD>
__device__ __attribute__((always_inline)) void amp_block(const float4* __restrict__ amp,
                                                      int64_t n_events, int64_t k0, int64_t k1,
                          int W, int lq, const double* __restrict__ v, double* __restrict__ rec)
{
    __shared__ double s_red[kAmpBlockWaves][64 * (WL + 1)];
    __shared__ double s_tot[kAmpBlockWaves][2 * 16 * WL];
    __shared__ double s_misc[kAmpBlockWaves][2];
    __shared__ double2 s_v[16 * WL];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwaves = blockDim.x >> 6;
    const int q = 1 << lq;
    const int sub = lane & (q - 1);

    for (int a = threadIdx.x; a < (WL << lq); a += blockDim.x)
        s_v[a] = a < W ? make_double2(v[2 * a], v[2 * a + 1]) : make_double2(0.0, 0.0);
    __syncthreads();
    AmpLane<WL> st;
    st.v = s_v + sub * WL;
#pragma unroll
    for (int k = 0; k < WL; ++k) {
        st.gr[k] = 0.0;
        st.gi[k] = 0.0;
    }
    st.dsum = 0.0;
    st.held = 1.0;
    st.nbad = 0;

    // this wavefront's steps: k0 + wave, k0 + wave + nwaves, ... (the block's
    // wavefronts stream its range together); the run position of the held
    // intensities counts the wavefront's own steps (every lane of an event
    // holds the same I, so any lane may keep it)
    const int64_t n_steps = k1 - k0;
    const int64_t J = n_steps > wave ? (n_steps - wave + nwaves - 1) / nwaves : 0;
    if (J > 0) {
        constexpr int64_t kStepVecs = 32 * WL;   // 64 lanes x WL / 2 vectors
        const float4* base = amp + lane;
        const int R_shift = 6 - lq;
        auto kof = [&](int64_t j) { return k0 + wave + (int64_t)nwaves * j; };
        AmpRegs<WL> ra, rb;
        amp_load(ra, base + kof(0) * kStepVecs);
        // No load is under a test: past the last step a load reads the step
        // just loaded again (cached; it is not used).  A load under a test
        // made the compiler copy its registers at the join, which waited for
        // the load it had just issued; now each step waits only for its own
        // buffer while the other buffer's loads stay in flight.
        for (int64_t j = 0; j < J; j += 2) {
            const bool has_b = j + 1 < J;
            const int64_t j1 = has_b ? j + 1 : j;
            amp_load(rb, base + kof(j1) * kStepVecs);
            amp_step<WL, GRAD>(ra, st, (kof(j) << R_shift) + (lane >> lq), n_events, lq, sub,
                               (int)(j & (q - 1)));
            const int64_t j2 = j + 2 < J ? j + 2 : j1;
            amp_load(ra, base + kof(j2) * kStepVecs);
            if (has_b)
                amp_step<WL, GRAD>(rb, st, (kof(j + 1) << R_shift) + (lane >> lq), n_events, lq,
                                   sub, (int)((j + 1) & (q - 1)));
        }
        st.dsum += log(st.held);   // a run cut short by the end of the range
    }

    const double dsum = wave_allsum(st.dsum);
    const int nbad = wave_allsum_int(st.nbad);
    if (lane == 0) {
        s_misc[wave][0] = dsum;
        s_misc[wave][1] = (double)nbad;
    }
    if (GRAD) {
        // lanes of the same sub-lane index hold the same waves: sum them in
        // lane order, real parts then imaginary parts
        double* red = s_red[wave];
        const int n_out = WL << lq;   // padded row length
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) {
            wave_lds_sync();
#pragma unroll
            for (int k = 0; k < WL; ++k) red[lane * (WL + 1) + k] = ri ? st.gi[k] : st.gr[k];
            wave_lds_sync();
            for (int o = lane; o < n_out; o += 64) {
                const int s = o / WL, k = o - s * WL;
                double x = 0.0;
                for (int e = 0; e < (64 >> lq); ++e) x += red[((e << lq) + s) * (WL + 1) + k];
                s_tot[wave][2 * o + ri] = x;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double d = 0.0, b = 0.0;
        for (int w = 0; w < nwaves; ++w) {
            d += s_misc[w][0];
            b += s_misc[w][1];
        }
        rec[0] = d;
        rec[1] = b;
    }
    if (GRAD) {
        for (int o = threadIdx.x; o < 2 * W; o += blockDim.x) {
            double x = 0.0;
            for (int w = 0; w < nwaves; ++w) x += s_tot[w][o];
            rec[2 + o] = x;
        }
    }
}

template <int WL, bool GRAD>
__global__ __launch_bounds__(64 * kAmpBlockWaves) void k_amp_fused(
    const float4* __restrict__ amp, int64_t n_events, int64_t n_steps, int W, int lq, VParams vp,
    double* __restrict__ partials, int rec_len)
{
    const int64_t k0 = (int64_t)blockIdx.x * n_steps / gridDim.x;
    const int64_t k1 = (int64_t)(blockIdx.x + 1) * n_steps / gridDim.x;
    amp_block<WL, GRAD>(amp, n_events, k0, k1, W, lq, vsrc(vp),
                        partials + (int64_t)blockIdx.x * rec_len);
}

// ---- many evaluations, possibly of different models, in one launch --------
// Block u takes work unit u: steps [k0, k1) of job units[u].job, whose V is at
// params + job.v_off; its record is record u (stride rec_stride doubles).
template <int WL>
__global__ __launch_bounds__(64 * kAmpBlockWaves) void k_amp_multi(
    const MultiJob* __restrict__ jobs, const MultiUnit* __restrict__ units,
    const double* __restrict__ params, double* __restrict__ recs, int rec_stride, int unit_off)
{
    const int u_idx = unit_off + blockIdx.x;
    const MultiUnit u = units[u_idx];
    const MultiJob j = jobs[u.job];
    amp_block<WL, true>((const float4*)j.amp, j.n_events, u.k0, u.k1, j.W, j.lq,
                        params + j.v_off, recs + (int64_t)u_idx * rec_stride);
}

int amp_multi_class(int wl) { return wl / 2 - 1; }

template <int WL>
static hipError_t launch_multi_class(const MultiLaunch& ml, const MultiClass& k, hipStream_t s)
{
    hipLaunchKernelGGL((k_amp_multi<WL>), dim3(k.n_units), dim3(64 * kAmpBlockWaves), 0, s,
                       ml.jobs, ml.units, ml.params, ml.recs, ml.rec_stride, k.unit_off);
    return hipGetLastError();
}

hipError_t launch_amp_multi_class(const MultiLaunch& ml, int c, hipStream_t s)
{
    const MultiClass& k = ml.cls[c];
    if (k.n_units == 0) return hipSuccess;
    switch (k.wl) {
    case 2: return launch_multi_class<2>(ml, k, s);
    case 4: return launch_multi_class<4>(ml, k, s);
    case 6: return launch_multi_class<6>(ml, k, s);
    case 8: return launch_multi_class<8>(ml, k, s);
    case 10: return launch_multi_class<10>(ml, k, s);
    case 12: return launch_multi_class<12>(ml, k, s);
    case 14: return launch_multi_class<14>(ml, k, s);
    case 16: return launch_multi_class<16>(ml, k, s);
    default: return hipErrorInvalidValue;
    }
}

template <int WL>
static int amp_grid_wl(const Model& m)
{
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)&k_amp_fused<WL, true>,
                                                     64 * kAmpBlockWaves, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int64_t n_steps = m.n_tiles << m.amp_lq;
    int64_t g = (int64_t)m.cus * per_cu;
    // at least 4 steps per wavefront
    const int64_t max_blocks = (n_steps + 4 * kAmpBlockWaves - 1) / (4 * kAmpBlockWaves);
    if (g > max_blocks) g = max_blocks;
    return (int)(g < 1 ? 1 : g);
}

int amp_fused_grid(Model& m)
{
    m.amp_waves = kAmpBlockWaves;
    switch (m.amp_wl) {
    case 2: return amp_grid_wl<2>(m);
    case 4: return amp_grid_wl<4>(m);
    case 6: return amp_grid_wl<6>(m);
    case 8: return amp_grid_wl<8>(m);
    case 10: return amp_grid_wl<10>(m);
    case 12: return amp_grid_wl<12>(m);
    case 14: return amp_grid_wl<14>(m);
    default: return amp_grid_wl<16>(m);
    }
}

template <int WL>
static hipError_t launch_amp_wl(const Model& m, const VParams& vp, bool grad, hipStream_t s,
                                const LaunchEvents& ev)
{
    const float4* a = (const float4*)m.d_data;
    const int64_t n_steps = m.n_tiles << m.amp_lq;
    const dim3 grid(m.grid), block(64 * kAmpBlockWaves);
    if (grad)
        hipExtLaunchKernelGGL((k_amp_fused<WL, true>), grid, block, 0, s, ev.start, ev.stop, 0, a,
                              m.n, n_steps, m.W, m.amp_lq, vp, m.d_partials, m.rec_len);
    else
        hipExtLaunchKernelGGL((k_amp_fused<WL, false>), grid, block, 0, s, ev.start, ev.stop, 0, a,
                              m.n, n_steps, m.W, m.amp_lq, vp, m.d_partials, m.rec_len);
    return hipGetLastError();
}

hipError_t launch_amp_fused(const Model& m, const VParams& vp, bool grad, hipStream_t s,
                            const LaunchEvents& ev)
{
    switch (m.amp_wl) {
    case 2: return launch_amp_wl<2>(m, vp, grad, s, ev);
    case 4: return launch_amp_wl<4>(m, vp, grad, s, ev);
    case 6: return launch_amp_wl<6>(m, vp, grad, s, ev);
    case 8: return launch_amp_wl<8>(m, vp, grad, s, ev);
    case 10: return launch_amp_wl<10>(m, vp, grad, s, ev);
    case 12: return launch_amp_wl<12>(m, vp, grad, s, ev);
    case 14: return launch_amp_wl<14>(m, vp, grad, s, ev);
    case 16: return launch_amp_wl<16>(m, vp, grad, s, ev);
    default: return hipErrorInvalidValue;
    }
}

// Lane-split complex64 copy of the amplitudes (complex128 input rounded to
// nearest); one thread per stored complex64, zero for padding.
__global__ void k_pack_amp(const void* __restrict__ src, bool c128, int64_t n, int W, int lq,
                           int wl, int64_t total, float2* __restrict__ dst)
{
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t f4 = g >> 1;                  // vector index
        const int64_t k = f4 / (32 * wl);           // step
        const int rem = (int)(f4 - k * (32 * wl));
        const int j = rem >> 6, lane = rem & 63;
        const int64_t i = (k << (6 - lq)) + (lane >> lq);
        const int a = (lane & ((1 << lq) - 1)) * wl + 2 * j + (int)(g & 1);
        float2 x = make_float2(0.f, 0.f);
        if (i < n && a < W) {
            if (c128) {
                const double2 d = reinterpret_cast<const double2*>(src)[i * W + a];
                x = make_float2((float)d.x, (float)d.y);
            } else {
                x = reinterpret_cast<const float2*>(src)[i * W + a];
            }
        }
        dst[g] = x;
    }
}

hipError_t launch_pack_amp(const void* src, bool src_c128, int64_t n, int W, AmpShape sh,
                           int64_t n_pad, float* dst, hipStream_t s)
{
    const int64_t total = n_pad * ((int64_t)sh.wl << sh.lq);
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_pack_amp, dim3((int)g), dim3(256), 0, s, src, src_c128, n, W, sh.lq,
                       sh.wl, total, (float2*)dst);
    return hipGetLastError();
}

// Row-major complex64 copy (N x W) of amplitudes stored in shape (lq, wl).
__global__ void k_unpack_amp(const float2* __restrict__ src, int64_t n, int W, int lq, int wl,
                             float2* __restrict__ dst)
{
    const int64_t total = n * W;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = g / W;
        const int a = (int)(g - i * W);
        const int64_t k = i >> (6 - lq);                       // step
        const int lane = ((int)(i & ((64 >> lq) - 1)) << lq) | (a / wl);
        const int kk = a % wl;
        dst[g] = src[((k * (wl / 2) + kk / 2) * 64 + lane) * 2 + (kk & 1)];
    }
}

hipError_t launch_unpack_amp(const void* src, int64_t n, int W, AmpShape sh, float* dst,
                             hipStream_t s)
{
    const int64_t total = n * W;
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_unpack_amp, dim3((int)g), dim3(256), 0, s, (const float2*)src, n, W,
                       sh.lq, sh.wl, (float2*)dst);
    return hipGetLastError();
}

}  // namespace pwa

namespace pwa {

// ---- FUMILI second derivatives (amplitude form) ----------------------------
// FUMILI takes, for the Hessian of -ln L, the sum over events of the outer
// products of the gradients of ln f; for the extended likelihood of Eq. 3 the
// dropped second derivatives of the data term cancel the MC term's Hessian on
// average, so the matrix is the data sum alone:
// H = sum_i J_i J_i^T over theta = (Re V_0, Im V_0, Re V_1, ...), with
// J_i = grad_theta ln I_i = 2 [Re z_ib, -Im z_ib]_b / I_i and z_ib = conj(S_i) A_ib
// (the derivative of Eq. 1).
//
// H = J^T J over the events is a matrix product with the events as its inner
// dimension: it runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64, D +=
// A B with A 16 x 4 and B 4 x 16).  The 2W parameters are cut into NB blocks
// of 16 (zero padded); a block pair (bp <= bq) accumulates
// D[i][j] = sum_k J_k[16 bp + i] J_k[16 bq + j].  Lane l of a wavefront takes
// event k = l / 16 of a step of 4 events and parameter i = l % 16 of every
// block: that is where both operands of the instruction expect J_k[16 b + i]
// (A[i][k] and B[k][j] sit in lane i + 16 k, D[4 r + l / 16][l % 16] in
// register r), so the J values a lane forms feed the matrix cores directly.
// Per block of 4 wavefronts, tiles of 64 events:
//   1. the tile's amplitudes into LDS, one row per event (de-interleaving the
//      lane-split layout), each row at least 8 NB entries long and zero past
//      the stored ones, so that no read of a row tests its index;
//   2. wavefront w takes events 16 w .. 16 w + 15: first S, I and w = 2 / I of
//      all 16 at once (lane l: event l % 16, a quarter of the waves, two xor
//      exchanges, then w S), then 4 steps of 4 events in which each lane
//      fetches its event's w S from the lane that formed it and forms its J
//      values in FP64;
//   3. one MFMA per block pair (bp of the block's group of rows, bq >= bp).
// Row groups: the block pairs of rows g R .. g R + R - 1 (R = NB up to 4 blocks,
// 2 up to 8, else 1) are one group along the grid's second dimension, each
// group streaming the tiles again.  The wavefronts are added in order through
// LDS; the record of a block column is [n_bad, then 256 doubles (a 16 x 16
// block, row-major) per block pair in packed order].  k_colsum adds the
// records column by column in a fixed order and k_hess_expand writes the
// matrix.  The next tile's amplitudes are loaded into registers while the
// current one is used.
constexpr int kHessThreads = 256;

__host__ __device__ inline int amp_lds_stride_words(int wpad)
{
    // 16-byte aligned rows whose word stride is 4 (mod 32): eight consecutive
    // lanes reading 16 bytes each cover all 32 banks.
    int words = 2 * wpad;
    int pad = ((4 - words) % 32 + 32) % 32;
    return words + pad;
}

__host__ __device__ inline int hess_nb(int W) { return (2 * W + 15) / 16; }
// Complex entries per LDS row of k_amp_hessian: at least 8 NB, so that
// parameter 16 b + i of every block reads entry (16 b + i) / 2 of its row; the
// entries past the stored wpad are zero.
__host__ __device__ inline int hess_row_waves(int wpad, int nb) { return wpad > 8 * nb ? wpad : 8 * nb; }
__host__ __device__ inline int hess_npair(int W)
{
    const int nb = hess_nb(W);
    return nb * (nb + 1) / 2;
}
__host__ __device__ inline int hess_rec_len(int W) { return 1 + 256 * hess_npair(W); }
__host__ __device__ constexpr int hess_rows_per_group(int nb) { return nb <= 4 ? nb : (nb <= 8 ? 2 : 1); }
inline int hess_groups(int W)
{
    const int nb = hess_nb(W);
    const int r = hess_rows_per_group(nb);
    return (nb + r - 1) / r;
}

template <int NB>
__host__ __device__ constexpr size_t hess_lds_bytes(int wpad)
{
    const size_t tile = (size_t)kAmpTile * amp_lds_stride_words(hess_row_waves(wpad, NB)) * 4;
    const size_t combine = (size_t)64 * hess_rows_per_group(NB) * NB * 4 * 8;
    return (tile > combine ? tile : combine) + 16 * 128 /* V */ + 16;
}

typedef double hd4 __attribute__((ext_vector_type(4)));

template <int NB>
__global__ __launch_bounds__(kHessThreads) void k_amp_hessian(const float4* __restrict__ amp,
                                                              int64_t n_events, int64_t n_tiles,
                                                              int W, int wpad, int lq, int wl,
                                                              VParams vp, double* __restrict__ recs)
{
    constexpr int R = hess_rows_per_group(NB);
    extern __shared__ double lds_d[];
    char* lds = reinterpret_cast<char*>(lds_d);
    const int row_waves = hess_row_waves(wpad, NB);
    const int stride = amp_lds_stride_words(row_waves) * 4;
    const size_t main_bytes = hess_lds_bytes<NB>(wpad) - 16 * 128 - 16;
    char* tile = lds;
    double2* s_v = reinterpret_cast<double2*>(lds + main_bytes);
    int* s_bad = reinterpret_cast<int*>(lds + main_bytes + 16 * 128);
    const int h = wpad >> 1;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int ki = lane >> 4;      // event of the step
    const int pi = lane & 15;      // parameter within a block
    // first row block of this group (known at compile time when one group
    // holds every row, so that only the upper block pairs take registers)
    const int g0 = R == NB ? 0 : (int)blockIdx.y * R;

    for (int a = tid; a < 128; a += blockDim.x)
        s_v[a] = a < W ? make_double2(vsrc(vp)[2 * a], vsrc(vp)[2 * a + 1]) : make_double2(0.0, 0.0);
    if (tid == 0) *s_bad = 0;
    // the row entries past the stored ones, read by the padding parameters
    // (staging never writes them; the loop's first barrier orders this)
    const int n_extra = row_waves - wpad;
    for (int e = tid; e < kAmpTile * n_extra; e += blockDim.x) {
        const int ev = e / n_extra, a = wpad + e % n_extra;
        *reinterpret_cast<float2*>(tile + ev * stride + a * 8) = make_float2(0.f, 0.f);
    }

    hd4 D[R][NB];
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
#pragma unroll
        for (int cq = 0; cq < NB; ++cq) D[rr][cq] = hd4{0.0, 0.0, 0.0, 0.0};
    int nbad = 0;

    const int64_t t0 = (int64_t)blockIdx.x * n_tiles / gridDim.x;
    const int64_t t1 = (int64_t)(blockIdx.x + 1) * n_tiles / gridDim.x;
    // the next tile's vectors are loaded into registers while the current one
    // is used, when a tile is at most PRE vectors per thread (rows of the
    // default shapes); otherwise they are staged directly
    constexpr int PRE = NB + 1;
    const int n_f4 = kAmpTile * h;
    const bool pre_ok = n_f4 <= PRE * kHessThreads;
    float4 pre[PRE];
    // lane-split layout -> one LDS row per event (16-byte column c)
    auto stage = [tile, stride, wl, lq](int f, float4 x) {
        const int kl = f / (32 * wl), rem = f - kl * 32 * wl;
        const int j = rem >> 6, ln = rem & 63;
        const int ev = (kl << (6 - lq)) + (ln >> lq);
        const int c = (ln & ((1 << lq) - 1)) * (wl >> 1) + j;
        *reinterpret_cast<float4*>(tile + ev * stride + c * 16) = x;
    };
    if (pre_ok && t0 < t1) {
        const float4* src = amp + t0 * kAmpTile * h;
#pragma unroll
        for (int q = 0; q < PRE; ++q) {
            const int f = tid + kHessThreads * q;
            pre[q] = f < n_f4 ? src[f] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
    for (int64_t t = t0; t < t1; ++t) {
        __syncthreads();   // the previous tile's rows are no longer read
        if (pre_ok) {
#pragma unroll
            for (int q = 0; q < PRE; ++q) {
                const int f = tid + kHessThreads * q;
                if (f < n_f4) stage(f, pre[q]);
            }
        } else {
            const float4* src = amp + t * kAmpTile * h;
            for (int f = tid; f < n_f4; f += blockDim.x) stage(f, src[f]);
        }
        __syncthreads();
        if (pre_ok && t + 1 < t1) {
            const float4* src = amp + (t + 1) * kAmpTile * h;
#pragma unroll
            for (int q = 0; q < PRE; ++q) {
                const int f = tid + kHessThreads * q;
                pre[q] = f < n_f4 ? src[f] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
        // S, I and w = 2 / I of this wavefront's 16 events, once per event:
        // lane l takes event l % 16 and the waves a = l / 16, l / 16 + 4, ...,
        // and two xor exchanges (lanes 16 and 32 apart) add the four quarters,
        // so every lane holds its event's S
        double esr = 0.0, esi = 0.0, ew = 0.0;
        {
            const int eg = lane & 15, aq = lane >> 4;
            const int ev = 16 * wave + eg;
            const char* row = tile + ev * stride;
            double sr = 0.0, si = 0.0;
            // every entry a < 8 NB of the row is stored or zero and V is zero
            // past W, so the loop runs to 8 NB without a test (the extra
            // terms add exact zeros) and its loads are issued together
#pragma unroll
            for (int m = 0; m < 2 * NB; ++m) {
                const int a = aq + 4 * m;
                const float2 x = *reinterpret_cast<const float2*>(row + a * 8);
                const double2 v = s_v[a];
                sr = __fma_rn(v.x, (double)x.x, sr);
                sr = __fma_rn(-v.y, (double)x.y, sr);
                si = __fma_rn(v.x, (double)x.y, si);
                si = __fma_rn(v.y, (double)x.x, si);
            }
            sr += xor_lane_f64<16>(sr);
            si += xor_lane_f64<16>(si);
            sr += xor_lane_f64<32>(sr);
            si += xor_lane_f64<32>(si);
            const double I = sr * sr + si * si;
            const bool valid = t * kAmpTile + ev < n_events;
            const bool ok = valid && (I > 0.0) && (I < INFINITY);
            if (aq == 0 && valid && !ok) ++nbad;
            // NaN for a degenerate event (its J, and so H, become NaN), 0 for padding
            ew = ok ? 2.0 * recip_f64(I) : (valid ? NAN : 0.0);
            esr = ew * sr;   // w Sr and w Si, the J coefficients of the event
            esi = ew * si;
        }
#pragma unroll 1
        for (int st = 0; st < 4; ++st) {
            const int ev = 16 * wave + 4 * st + ki;
            const char* row = tile + ev * stride;
            // this lane's event (4 st + ki of the wavefront's 16) from the
            // lane that formed it
            const int src = 4 * st + ki;
            const double wsr = __shfl(esr, src);
            const double wsi = __shfl(esi, src);
            // J_k[p] for parameter p = 16 b + pi: w Re z (p even) or -w Im z (p odd),
            // z = conj(S) A_{p / 2}: Re z = Sr Ar + Si Ai, -Im z = Si Ar - Sr Ai, so
            // J = c1 Ar + c2 Ai with a lane's (c1, c2) = (w Sr, w Si) or
            // (w Si, -w Sr) (the parity of p is the lane's)
            const double c1 = (pi & 1) ? wsi : wsr;
            const double c2 = (pi & 1) ? -wsr : wsi;
            // a parameter past 2W reads a zero entry of the row, so its J is
            // zero (NaN for a degenerate event, in rows and columns of the
            // block pairs that are never read); no load waits behind a branch
            auto jval = [&](int b) {
                const float2 x = *reinterpret_cast<const float2*>(row + (8 * b + (pi >> 1)) * 8);
                return __fma_rn(c1, (double)x.x, c2 * (double)x.y);
            };
            double Jv[NB];
#pragma unroll
            for (int cq = 0; cq < NB; ++cq) Jv[cq] = jval(cq);
#pragma unroll
            for (int rr = 0; rr < R; ++rr) {
                const int bp = g0 + rr;
                if (bp < NB) {
                    const double Jp = R == NB ? Jv[rr] : jval(bp);
#pragma unroll
                    for (int cq = 0; cq < NB; ++cq)
                        if (cq >= bp)
                            D[rr][cq] = __builtin_amdgcn_mfma_f64_16x16x4f64(Jp, Jv[cq], D[rr][cq],
                                                                             0, 0, 0);
                }
            }
        }
    }

    // n_bad: one lane per event counted; the block's total by LDS atomics
    nbad = wave_allsum_int(nbad);
    __syncthreads();
    if (lane == 0 && nbad) atomicAdd(s_bad, nbad);   // LDS, order-free integer count
    // the wavefronts' D added in wavefront order through LDS (the tile area)
    double* s_d = reinterpret_cast<double*>(lds);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        __syncthreads();
        if (wave == w) {
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
#pragma unroll
                for (int cq = 0; cq < NB; ++cq)
                    if (g0 + rr < NB && cq >= g0 + rr)
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            double* slot = s_d + ((size_t)((rr * NB + cq) * 4 + r) * 64 + lane);
                            *slot = (w == 0 ? 0.0 : *slot) + D[rr][cq][r];
                        }
        }
    }
    __syncthreads();
    double* rec = recs + (int64_t)blockIdx.x * hess_rec_len(W);
    // record: block pair (bp, bq) at 1 + 256 * pair, element [i][j] row-major,
    // from lane l = j + 16 (i % 4), register r = i / 4
    for (int rr = 0; rr < R; ++rr) {
        const int bp = g0 + rr;
        if (bp >= NB) break;
        for (int e = tid; e < (NB - bp) * 256; e += blockDim.x) {
            const int cq = bp + e / 256, ij = e % 256;
            const int i = ij >> 4, j = ij & 15;
            const int l = j + 16 * (i & 3), r = i >> 2;
            const int pair = bp * NB - bp * (bp - 1) / 2 + (cq - bp);
            rec[1 + (size_t)pair * 256 + ij] = s_d[(size_t)((rr * NB + cq) * 4 + r) * 64 + l];
        }
    }
    if (tid == 0 && blockIdx.y == 0) rec[0] = (double)*s_bad;
}

// Wider rows (NB > 4 blocks, W > 32): the block pairs no longer fit one
// wavefront's registers, and repeating the pass per row group re-reads the
// amplitudes and re-forms J every time.  Instead a block of 16 wavefronts
// (one per CU) forms J once per event into LDS and each wavefront owns a fixed
// range of at most ceil(pairs / 16) block pairs, indexed at run time
// (wavefront-uniform, scalar registers) so that one code path serves every
// wavefront within the 128 registers of a 1024-thread block:
//   1. the tile's amplitudes into LDS, one row per event (as above);
//   2. per half tile of 32 events: wavefront w takes events 2w and 2w + 1,
//      32 lanes each; S over waves pi, pi + 32, ... and an xor butterfly
//      over the 32 lanes, then w = 2 / I and J_p for p = pi + 32 m into an
//      LDS row of 16 NB doubles (zero beyond 2W, or NaN for a degenerate
//      event, in rows and columns of the blocks that are never read); the
//      amplitude rows hold hess_wide_row_waves entries, those past the stored
//      wpad zero, so that neither loop tests its index against W;
//   3. per step of 4 events, one MFMA per owned pair with both operands read
//      from the J rows (lane l: event l / 16 of the step, parameter l % 16).
// Each pair has one owner, which writes its 16 x 16 block straight into the
// block's record (same layout as above; row groups are not used).
constexpr int kHessWideWaves = 16;
constexpr int kHessWideHalf = 32;   // events per J stage

// Complex entries per amplitude row of the wide kernel (wpad <= 8 NB): a
// multiple of 32, so that lane pi of the S loop reads pi + 32 m for a fixed
// count of m.
__host__ __device__ constexpr int hess_wide_row_waves(int nb) { return 32 * ((8 * nb + 31) / 32); }

__host__ __device__ inline size_t hess_wide_lds_bytes(int wpad, int nb)
{
    (void)wpad;
    return (size_t)kAmpTile * amp_lds_stride_words(hess_wide_row_waves(nb)) * 4   // amplitude rows
           + (size_t)kHessWideHalf * 16 * nb * 8                    // J rows
           + 16 * 128 /* V */ + 16;
}

template <int NB>
__global__ __launch_bounds__(64 * kHessWideWaves) void k_amp_hessian_wide(
    const float4* __restrict__ amp, int64_t n_events, int64_t n_tiles, int W, int wpad, int lq,
    int wl, VParams vp, double* __restrict__ recs)
{
    constexpr int NT = 64 * kHessWideWaves;
    constexpr int NPAIR = NB * (NB + 1) / 2;
    constexpr int PPW = (NPAIR + kHessWideWaves - 1) / kHessWideWaves;
    constexpr int XW = 16 * NB;                       // J row (doubles)
    constexpr int PRE = (kAmpTile * 8 * NB / 2 + NT - 1) / NT;   // float4 per thread (wpad <= 8 NB)
    constexpr int RW = hess_wide_row_waves(NB);
    extern __shared__ double lds_d[];
    char* lds = reinterpret_cast<char*>(lds_d);
    const int stride = amp_lds_stride_words(RW) * 4;
    char* tile = lds;
    double* s_j = reinterpret_cast<double*>(lds + (size_t)kAmpTile * stride);
    double2* s_v = reinterpret_cast<double2*>(lds + (size_t)kAmpTile * stride +
                                              (size_t)kHessWideHalf * XW * 8);
    int* s_bad = reinterpret_cast<int*>(s_v + 128);
    const int h = wpad >> 1;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    for (int a = tid; a < 128; a += NT)
        s_v[a] = a < W ? make_double2(vsrc(vp)[2 * a], vsrc(vp)[2 * a + 1]) : make_double2(0.0, 0.0);
    if (tid == 0) *s_bad = 0;
    // the row entries past the stored ones (staging never writes them; the
    // loop's first barrier orders this)
    const int n_extra = RW - wpad;
    for (int e = tid; e < kAmpTile * n_extra; e += NT) {
        const int ev = e / n_extra, a = wpad + e % n_extra;
        *reinterpret_cast<float2*>(tile + ev * stride + a * 8) = make_float2(0.f, 0.f);
    }

    // this wavefront's block pairs (bp <= bq, row-major), as column offsets
    int pt[PPW], pu[PPW];
#pragma unroll
    for (int pp = 0; pp < PPW; ++pp) {
        int p = wave * PPW + pp, t = 0;
        if (p >= NPAIR) p = NPAIR - 1;   // past the last pair: never used
        while (p >= NB - t) {
            p -= NB - t;
            ++t;
        }
        pt[pp] = __builtin_amdgcn_readfirstlane(16 * t);
        pu[pp] = __builtin_amdgcn_readfirstlane(16 * (t + p));
    }
    const int n_mine = min(PPW, max(0, NPAIR - wave * PPW));
    hd4 D[PPW];
#pragma unroll
    for (int pp = 0; pp < PPW; ++pp) D[pp] = hd4{0.0, 0.0, 0.0, 0.0};
    int nbad = 0;

    const int64_t t0 = (int64_t)blockIdx.x * n_tiles / gridDim.x;
    const int64_t t1 = (int64_t)(blockIdx.x + 1) * n_tiles / gridDim.x;
    const int n_f4 = kAmpTile * h;
    float4 pre[PRE];
    auto stage = [tile, stride, wl, lq](int f, float4 x) {
        const int kl = f / (32 * wl), rem = f - kl * 32 * wl;
        const int j = rem >> 6, ln = rem & 63;
        const int ev = (kl << (6 - lq)) + (ln >> lq);
        const int c = (ln & ((1 << lq) - 1)) * (wl >> 1) + j;
        *reinterpret_cast<float4*>(tile + ev * stride + c * 16) = x;
    };
    auto load_tile = [&](int64_t t) {
        const float4* src = amp + t * kAmpTile * h;
#pragma unroll
        for (int q = 0; q < PRE; ++q) {
            const int f = tid + NT * q;
            pre[q] = f < n_f4 ? src[f] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    if (t0 < t1) load_tile(t0);
    const int ke = lane >> 5;    // J stage: event of the wavefront's pair
    const int pj = lane & 31;    // J stage: lane within the event
    const int k = lane >> 4;     // MFMA: event of the step
    const int i = lane & 15;     // MFMA: parameter within a block
    for (int64_t t = t0; t < t1; ++t) {
        __syncthreads();   // the previous tile's rows and J are no longer read
#pragma unroll
        for (int q = 0; q < PRE; ++q) {
            const int f = tid + NT * q;
            if (f < n_f4) stage(f, pre[q]);
        }
        __syncthreads();
        if (t + 1 < t1) load_tile(t + 1);
        for (int half = 0; half < kAmpTile / kHessWideHalf; ++half) {
            // 2. J of events 2 wave + ke of this half
            {
                const int eh = 2 * wave + ke;                 // event within the half
                const int ev = kHessWideHalf * half + eh;     // event within the tile
                const char* row = tile + ev * stride;
                double sr = 0.0, si = 0.0;
                // entries up to RW are stored or zero and V is zero past W:
                // no test, the loads issued together, the extra terms zero
#pragma unroll
                for (int m = 0; m < RW / 32; ++m) {
                    const int a = pj + 32 * m;
                    const float2 x = *reinterpret_cast<const float2*>(row + a * 8);
                    const double2 v = s_v[a];
                    sr = __fma_rn(v.x, (double)x.x, sr);
                    sr = __fma_rn(-v.y, (double)x.y, sr);
                    si = __fma_rn(v.x, (double)x.y, si);
                    si = __fma_rn(v.y, (double)x.x, si);
                }
                sr += xor_lane_f64<1>(sr);
                si += xor_lane_f64<1>(si);
                sr += xor_lane_f64<2>(sr);
                si += xor_lane_f64<2>(si);
                sr += xor_lane_f64<4>(sr);
                si += xor_lane_f64<4>(si);
                sr += xor_lane_f64<8>(sr);
                si += xor_lane_f64<8>(si);
                sr += xor_lane_f64<16>(sr);
                si += xor_lane_f64<16>(si);
                const double I = sr * sr + si * si;
                const bool valid = t * kAmpTile + ev < n_events;
                const bool ok = valid && (I > 0.0) && (I < INFINITY);
                if (pj == 0 && valid && !ok) ++nbad;
                // NaN for a degenerate event (its J, and so H, become NaN), 0 for padding
                const double w = ok ? 2.0 * recip_f64(I) : (valid ? NAN : 0.0);
                // J = c1 Re A + c2 Im A (the parity of p = pj + 32 m is the lane's)
                const double c1 = w * ((pj & 1) ? si : sr);
                const double c2 = w * ((pj & 1) ? -sr : si);
                double* jrow = s_j + eh * XW;
                // a parameter past 2W reads a zero entry (p / 2 < 8 NB <= RW)
#pragma unroll
                for (int m = 0; m < XW / 32; ++m) {
                    const int p = pj + 32 * m;
                    const float2 x = *reinterpret_cast<const float2*>(row + (p >> 1) * 8);
                    jrow[p] = __fma_rn(c1, (double)x.x, c2 * (double)x.y);
                }
                if constexpr (XW % 32 != 0) {
                    const int p = pj + 32 * (XW / 32);
                    if (p < XW) {
                        const float2 x = *reinterpret_cast<const float2*>(row + (p >> 1) * 8);
                        jrow[p] = __fma_rn(c1, (double)x.x, c2 * (double)x.y);
                    }
                }
            }
            __syncthreads();
            // 3. the owned block pairs over the half's 8 steps, one at a time
            // (unrolled, the scheduler hoists later steps' loads past the 128
            // registers and spills)
#pragma unroll 1
            for (int st = 0; st < kHessWideHalf / 4; ++st) {
                const double* jr = s_j + (4 * st + k) * XW + i;
#pragma unroll
                for (int pp = 0; pp < PPW; ++pp)
                    if (pp < n_mine)
                        D[pp] = __builtin_amdgcn_mfma_f64_16x16x4f64(jr[pt[pp]], jr[pu[pp]], D[pp],
                                                                     0, 0, 0);
            }
            __syncthreads();   // J rows free for the next half
        }
    }

    nbad = wave_allsum_int(nbad);
    if (lane == 0 && nbad) atomicAdd(s_bad, nbad);   // LDS, order-free integer count
    double* rec = recs + (int64_t)blockIdx.x * hess_rec_len(W);
    // element [i][j] of a pair's block is in lane j + 16 (i % 4), register i / 4
#pragma unroll
    for (int pp = 0; pp < PPW; ++pp)
        if (pp < n_mine)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                rec[1 + (size_t)(wave * PPW + pp) * 256 + 16 * (4 * r + (lane >> 4)) + (lane & 15)] =
                    D[pp][r];
    __syncthreads();
    if (tid == 0) rec[0] = (double)*s_bad;
}

// The matrix from the column sums of the block records (k_colsum: one
// wavefront per column, fixed order); one thread per entry of the 2W x 2W
// matrix (full, row-major), written to pinned host memory.
__global__ __launch_bounds__(256) void k_hess_expand(const double* __restrict__ colsum, int W,
                                                     double* out, unsigned long long* done,
                                                     unsigned long long seq)
{
    const int P = 2 * W;
    const int nb = hess_nb(W);
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < P * P) {
        int p = e / P, q = e % P;
        if (p > q) {   // the lower triangle mirrors the upper
            const int tp = p;
            p = q;
            q = tp;
        }
        const int i = p / 16, j = q / 16;
        const int pair = i * nb - i * (i - 1) / 2 + (j - i);
        const double x = colsum[1 + pair * 256 + 16 * (p % 16) + (q % 16)];
        store_system(out + e, colsum[0] > 0.0 ? NAN : x);
    }
    wait_vm_complete();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(done + blockIdx.x, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// block columns: fewer when the row groups multiply the blocks; one
// 16-wavefront block per CU for the wide rows (then also the row-group
// kernel's column count, so that the record buffer never depends on the shape)
int hess_grid(const Model& m)
{
    if (hess_nb(m.W) > 4)
        return (int)std::min<int64_t>(m.cus, std::max<int64_t>(1, m.n_tiles));
    const int64_t want = std::max<int64_t>(64, 4 * (int64_t)m.cus / hess_groups(m.W));
    return (int)std::min<int64_t>(want, std::max<int64_t>(1, m.n_tiles));
}
// block records plus one row for their column sums
int hess_rows(const Model& m) { return hess_grid(m) + 1; }
int hess_rec_doubles(int W) { return hess_rec_len(W); }
int hess_assemble_blocks(int W) { return (4 * W * W + 255) / 256; }

template <int NB>
static hipError_t launch_hessian_nb(const Model& m, const VParams& vp, double* recs, hipStream_t s)
{
    // the wide kernel when the stored rows are no wider than its staging
    // assumes (every default or tuned shape; a shape set by hand may pad more)
    if constexpr (NB > 4) {
        if (m.wpad <= 8 * NB && hess_wide_lds_bytes(m.wpad, NB) <= kLdsBytes) {
            const size_t lds = hess_wide_lds_bytes(m.wpad, NB);
            const hipError_t e = hipFuncSetAttribute((const void*)&k_amp_hessian_wide<NB>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_amp_hessian_wide<NB>), dim3(hess_grid(m)),
                               dim3(64 * kHessWideWaves), lds, s, (const float4*)m.d_data, m.n,
                               m.n_tiles, m.W, m.wpad, m.amp_lq, m.amp_wl, vp, recs);
            return hipGetLastError();
        }
    }
    const size_t lds = hess_lds_bytes<NB>(m.wpad);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void*)&k_amp_hessian<NB>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_amp_hessian<NB>), dim3(hess_grid(m), hess_groups(m.W)),
                       dim3(kHessThreads), lds, s, (const float4*)m.d_data, m.n, m.n_tiles, m.W,
                       m.wpad, m.amp_lq, m.amp_wl, vp, recs);
    return hipGetLastError();
}

hipError_t launch_hessian(const Model& m, const VParams& vp, double* recs, double* out,
                          unsigned long long* done, unsigned long long seq, hipStream_t s)
{
    hipError_t e = hipErrorInvalidValue;
    switch (hess_nb(m.W)) {
    case 1: e = launch_hessian_nb<1>(m, vp, recs, s); break;
    case 2: e = launch_hessian_nb<2>(m, vp, recs, s); break;
    case 3: e = launch_hessian_nb<3>(m, vp, recs, s); break;
    case 4: e = launch_hessian_nb<4>(m, vp, recs, s); break;
    case 5: e = launch_hessian_nb<5>(m, vp, recs, s); break;
    case 6: e = launch_hessian_nb<6>(m, vp, recs, s); break;
    case 7: e = launch_hessian_nb<7>(m, vp, recs, s); break;
    case 8: e = launch_hessian_nb<8>(m, vp, recs, s); break;
    case 9: e = launch_hessian_nb<9>(m, vp, recs, s); break;
    case 10: e = launch_hessian_nb<10>(m, vp, recs, s); break;
    case 11: e = launch_hessian_nb<11>(m, vp, recs, s); break;
    case 12: e = launch_hessian_nb<12>(m, vp, recs, s); break;
    case 13: e = launch_hessian_nb<13>(m, vp, recs, s); break;
    case 14: e = launch_hessian_nb<14>(m, vp, recs, s); break;
    case 15: e = launch_hessian_nb<15>(m, vp, recs, s); break;
    case 16: e = launch_hessian_nb<16>(m, vp, recs, s); break;
    default: break;
    }
    if (e != hipSuccess) return e;
    const int rows = hess_grid(m), rl = hess_rec_len(m.W);
    double* colsum = recs + (size_t)rows * rl;
    e = launch_colsum(recs, rows, rl, rl, colsum, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hess_expand, dim3(hess_assemble_blocks(m.W)), dim3(256), 0, s, colsum,
                       m.W, out, done, seq);
    return hipGetLastError();
}

}  // namespace pwa
