// k_amp.hip -- amplitude-form NLL + gradient (Eq. 1 inside Eq. 3): the
// per-event work is S_i = sum_a V_a A_ia and I_i = |S_i|^2, so only N x W
// amplitudes are streamed instead of the N x W(W+1)/2 table.
//
// Amplitudes are stored complex64, row-major, each row padded to an even
// number of waves wpad and the event count padded to a multiple of 64 with
// zero rows.  A block has up to four wavefronts; each handles tiles of 64 events:
//   1. coalesced 16-byte loads of the tile's contiguous 512*wpad bytes into LDS
//      (rows padded in LDS so that the per-event reads below hit distinct banks);
//   2. lane = event: S_i, I_i, ln I_i and c_i = S_i / I_i in FP64;
//   3. g_a += c_i conj(A_ia) over the tile's 64 events, reading the tile from
//      LDS (so the amplitudes leave HBM once per evaluation): for W <= 64 the
//      lanes are G = 64 / W groups of W, group q taking events q, q + G, ...,
//      and the groups are added in order at the end; beyond 64 waves,
//      lane = wave.
// Each block writes one partial record [sum ln I, n_bad, g_0, ..., g_{W-1}];
// the gradient is G_b = 2 sum_a V_a M_ab - 2 g_b.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pwa_internal.h"
#include "tail.h"
#include "wave_ops.h"

namespace pwa {

__host__ __device__ inline int amp_lds_stride_words(int wpad)
{
    // 16-byte aligned rows whose word stride is 4 (mod 32): eight consecutive
    // lanes reading 16 bytes each cover all 32 banks.
    int words = 2 * wpad;
    int pad = ((4 - words) % 32 + 32) % 32;
    return words + pad;
}

// LDS of one wavefront: its tile of kAmpTile rows and the per-event weights.
__host__ __device__ inline size_t amp_wave_lds_bytes(int wpad)
{
    return (size_t)kAmpTile * amp_lds_stride_words(wpad) * 4 + kAmpTile * 16;
}

__host__ __device__ inline size_t amp_lds_bytes(int wpad, int nwaves)
{
    const size_t main = (size_t)wpad * 16 + nwaves * amp_wave_lds_bytes(wpad);
    const size_t combine = (size_t)wpad * 16 + 2 * 64 * 16 + 16;   // wave combine at the end
    return main > combine ? main : combine;
}

// Wavefronts per block: four unless their tiles would not fit twice per CU.
inline int amp_waves_per_block(int wpad)
{
    int w = 4;
    while (w > 1 && amp_lds_bytes(wpad, w) > 80 * 1024) w >>= 1;
    return w;
}

// One block's share: tiles [t0, t1) of one evaluation, V (2W doubles) from
// `v`, one record [sum ln I, n_bad, g_0, ..., g_{W-1}] to `rec`.
template <int KW, bool GRAD>
__device__ void amp_block(const float4* __restrict__ amp, int64_t n_events, int64_t t0,
                          int64_t t1, int W, int wpad, const double* __restrict__ v,
                          double* __restrict__ rec)
{
    extern __shared__ double lds_d[];
    char* lds = reinterpret_cast<char*>(lds_d);
    const int stride = amp_lds_stride_words(wpad) * 4;      // bytes per LDS row
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwaves = blockDim.x >> 6;
    double2* s_v = reinterpret_cast<double2*>(lds);
    char* tile = lds + (size_t)wpad * 16 + (size_t)wave * amp_wave_lds_bytes(wpad);
    double2* s_cw = reinterpret_cast<double2*>(tile + kAmpTile * stride);
    const int h = wpad >> 1;                                 // 16-byte vectors per row

    for (int a = threadIdx.x; a < wpad; a += blockDim.x)
        s_v[a] = (a < W) ? make_double2(v[2 * a], v[2 * a + 1]) : make_double2(0.0, 0.0);
    __syncthreads();

    double gr[KW], gi[KW];
#pragma unroll
    for (int s = 0; s < KW; ++s) { gr[s] = 0.0; gi[s] = 0.0; }
    double dsum = 0.0;
    int nbad = 0;
    // adjoint lane mapping for W <= 64: G = 64 / W event groups of W lanes
    const int G = KW == 1 ? 64 / W : 1;
    const int a_lane = KW == 1 ? lane % W : lane;
    const int grp = KW == 1 ? lane / W : 0;

    // the block's tiles, interleaved over its wavefronts; each wavefront uses
    // only its own LDS region, so it synchronises with itself only
    for (int64_t t = t0 + wave; t < t1; t += nwaves) {
        const float4* src = amp + t * kAmpTile * h;
        for (int q = 0; q < h; ++q) {
            const int f = q * 64 + lane;
            const float4 val = src[f];
            const int ev = f / h;
            const int c = f - ev * h;
            *reinterpret_cast<float4*>(tile + ev * stride + c * 16) = val;
        }
        wave_lds_sync();

        // lane = event
        const char* row = tile + lane * stride;
        double sr = 0.0, si = 0.0;
        for (int c = 0; c < h; ++c) {
            const float4 x = *reinterpret_cast<const float4*>(row + c * 16);
            const double2 v0 = s_v[2 * c], v1 = s_v[2 * c + 1];
            sr += v0.x * (double)x.x - v0.y * (double)x.y;
            si += v0.x * (double)x.y + v0.y * (double)x.x;
            sr += v1.x * (double)x.z - v1.y * (double)x.w;
            si += v1.x * (double)x.w + v1.y * (double)x.z;
        }
        const double I = sr * sr + si * si;
        const bool valid = t * kAmpTile + lane < n_events;
        const bool ok = valid && (I > 0.0) && (I < INFINITY);
        if (ok) dsum += log(I);
        if (valid && !ok) ++nbad;
        if (GRAD) {
            // NaN for a degenerate event (the gradient becomes NaN), 0 for padding
            const double w = ok ? 1.0 / I : (valid ? NAN : 0.0);
            s_cw[lane] = make_double2(w * sr, w * si);
            wave_lds_sync();
            if (KW == 1) {
                // lane = (wave a, event group grp): events grp, grp + G, ...,
                // four at a time with separate partial sums so that the LDS
                // reads are in flight together
                if (grp < G) {   // the 64 - G W lanes beyond the groups idle
                    double pr[4] = {0.0, 0.0, 0.0, 0.0}, pi[4] = {0.0, 0.0, 0.0, 0.0};
                    int l = grp;
                    for (; l + 3 * G < kAmpTile; l += 4 * G) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const double2 c = s_cw[l + q * G];
                            const float2 x = *reinterpret_cast<const float2*>(
                                tile + (l + q * G) * stride + a_lane * 8);
                            pr[q] += c.x * (double)x.x + c.y * (double)x.y;
                            pi[q] += c.y * (double)x.x - c.x * (double)x.y;
                        }
                    }
                    for (; l < kAmpTile; l += G) {
                        const double2 c = s_cw[l];
                        const float2 x =
                            *reinterpret_cast<const float2*>(tile + l * stride + a_lane * 8);
                        pr[0] += c.x * (double)x.x + c.y * (double)x.y;
                        pi[0] += c.y * (double)x.x - c.x * (double)x.y;
                    }
                    gr[0] += (pr[0] + pr[1]) + (pr[2] + pr[3]);
                    gi[0] += (pi[0] + pi[1]) + (pi[2] + pi[3]);
                }
            } else {
                // lane = wave (two per lane beyond 64 waves)
                for (int l = 0; l < kAmpTile; ++l) {
                    const double2 c = s_cw[l];
                    const float2* rl = reinterpret_cast<const float2*>(tile + l * stride);
#pragma unroll
                    for (int s = 0; s < KW; ++s) {
                        const int a = lane + 64 * s;
                        if (a < W) {
                            const float2 x = rl[a];
                            gr[s] += c.x * (double)x.x + c.y * (double)x.y;
                            gi[s] += c.y * (double)x.x - c.x * (double)x.y;
                        }
                    }
                }
            }
        }
        wave_lds_sync();
    }

    // combine the block's wavefronts in a fixed order (reusing wave 0's tile)
    dsum = wave_allsum(dsum);
    nbad = wave_allsum_int(nbad);
    if (KW == 1 && GRAD) {
        // fold the event groups of each wave a into lane a, in group order,
        // through this wavefront's own tile region
        double2* s_fold = reinterpret_cast<double2*>(tile);
        wave_lds_sync();
        s_fold[lane] = make_double2(gr[0], gi[0]);
        wave_lds_sync();
        if (lane < W) {
            double xr = 0.0, xi = 0.0;
            for (int q = 0; q < G; ++q) {
                xr += s_fold[q * W + lane].x;
                xi += s_fold[q * W + lane].y;
            }
            gr[0] = xr;
            gi[0] = xi;
        } else {
            gr[0] = 0.0;
            gi[0] = 0.0;
        }
        wave_lds_sync();
    }
    __syncthreads();
    double2* s_g = reinterpret_cast<double2*>(lds + (size_t)wpad * 16);
    double* s_misc = reinterpret_cast<double*>(s_g + 2 * 64);   // after KW <= 2 slots of 64
    for (int w = 0; w < nwaves; ++w) {
        if (wave == w) {
#pragma unroll
            for (int s = 0; s < KW; ++s) {
                double2 g = make_double2(gr[s], gi[s]);
                if (w > 0) {
                    const double2 o = s_g[s * 64 + lane];
                    g.x += o.x;
                    g.y += o.y;
                }
                s_g[s * 64 + lane] = g;
            }
            if (lane == 0) {
                s_misc[0] = (w > 0 ? s_misc[0] : 0.0) + dsum;
                s_misc[1] = (w > 0 ? s_misc[1] : 0.0) + (double)nbad;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        rec[0] = s_misc[0];
        rec[1] = s_misc[1];
    }
    if (GRAD) {
        for (int a = threadIdx.x; a < W; a += blockDim.x) {
            rec[2 + 2 * a] = s_g[a].x;
            rec[3 + 2 * a] = s_g[a].y;
        }
    }
}

template <int KW, bool GRAD>
__global__ __launch_bounds__(256) void k_amp_fused(const float4* __restrict__ amp, int64_t n_events,
                                                   int64_t n_tiles, int W, int wpad, VParams vp,
                                                   double* __restrict__ partials, int rec_len)
{
    const int64_t t0 = (int64_t)blockIdx.x * n_tiles / gridDim.x;
    const int64_t t1 = (int64_t)(blockIdx.x + 1) * n_tiles / gridDim.x;
    amp_block<KW, GRAD>(amp, n_events, t0, t1, W, wpad, vp.v,
                        partials + (int64_t)blockIdx.x * rec_len);
}

// ---- many evaluations, possibly of different models, in one launch --------
// Block u takes work unit u: tiles [t0, t1) of job units[u].job, whose V is at
// params + job.v_off; its record is record u (stride rec_stride doubles).
template <int KW>
__global__ __launch_bounds__(256) void k_amp_multi(const MultiJob* __restrict__ jobs,
                                                   const MultiUnit* __restrict__ units,
                                                   const double* __restrict__ params,
                                                   double* __restrict__ recs, int rec_stride,
                                                   int unit_off)
{
    const int u_idx = unit_off + blockIdx.x;
    const MultiUnit u = units[u_idx];
    const MultiJob j = jobs[u.job];
    amp_block<KW, true>((const float4*)j.amp, j.n_events, u.t0, u.t1, j.W, j.wpad,
                        params + j.v_off, recs + (int64_t)u_idx * rec_stride);
}

// width classes: rows of at most 16, 32, 48, 64 and 128 waves
int amp_multi_class(int wpad)
{
    return wpad <= 16 ? 0 : wpad <= 32 ? 1 : wpad <= 48 ? 2 : wpad <= 64 ? 3 : 4;
}

hipError_t launch_amp_multi(const MultiLaunch& ml, hipStream_t s)
{
    for (int c = 0; c < ml.n_classes; ++c) {
        const MultiClass& k = ml.cls[c];
        if (k.n_units == 0) continue;
        const int waves = amp_waves_per_block(k.wpad);
        const size_t lds = amp_lds_bytes(k.wpad, waves);
        const dim3 grid(k.n_units), block(64 * waves);
        if (k.wpad <= 64)
            hipLaunchKernelGGL((k_amp_multi<1>), grid, block, lds, s, ml.jobs, ml.units, ml.params,
                               ml.recs, ml.rec_stride, k.unit_off);
        else
            hipLaunchKernelGGL((k_amp_multi<2>), grid, block, lds, s, ml.jobs, ml.units, ml.params,
                               ml.recs, ml.rec_stride, k.unit_off);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int amp_multi_waves(int wpad) { return amp_waves_per_block(wpad); }

hipError_t amp_multi_prepare(int wpad)
{
    const size_t lds = amp_lds_bytes(wpad, amp_waves_per_block(wpad));
    if (lds > 65536) {
        const void* fns[] = {(const void*)&k_amp_multi<1>, (const void*)&k_amp_multi<2>};
        for (const void* f : fns) {
            const hipError_t e =
                hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

template <int KW>
static const void* amp_symbol()
{
    return (const void*)&k_amp_fused<KW, true>;
}

int amp_fused_grid(Model& m)
{
    const int nw = amp_waves_per_block(m.wpad);
    m.amp_waves = nw;
    const void* fn = (m.wpad <= 64) ? amp_symbol<1>() : amp_symbol<2>();
    const size_t lds = amp_lds_bytes(m.wpad, nw);
    if (lds > 65536) {
        // wide rows: allow more than the default 64 KB of dynamic LDS
        const void* fns[] = {(const void*)&k_amp_fused<1, true>, (const void*)&k_amp_fused<1, false>,
                             (const void*)&k_amp_fused<2, true>, (const void*)&k_amp_fused<2, false>};
        for (const void* f : fns)
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * nw, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int64_t g = (int64_t)m.cus * per_cu;
    const int64_t max_blocks = (m.n_tiles + nw - 1) / nw;
    if (g > max_blocks) g = max_blocks;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_amp_fused(const Model& m, const VParams& vp, bool grad, hipStream_t s,
                            const LaunchEvents& ev)
{
    const int nw = m.amp_waves;
    const size_t lds = amp_lds_bytes(m.wpad, nw);
    const float4* a = (const float4*)m.d_data;
    const dim3 grid(m.grid), block(64 * nw);
    const hipEvent_t t0 = ev.start, t1 = ev.stop;
    if (m.wpad <= 64) {
        if (grad)
            hipExtLaunchKernelGGL((k_amp_fused<1, true>), grid, block, lds, s, t0, t1, 0, a, m.n,
                                  m.n_tiles, m.W, m.wpad, vp, m.d_partials, m.rec_len);
        else
            hipExtLaunchKernelGGL((k_amp_fused<1, false>), grid, block, lds, s, t0, t1, 0, a, m.n,
                                  m.n_tiles, m.W, m.wpad, vp, m.d_partials, m.rec_len);
    } else {
        if (grad)
            hipExtLaunchKernelGGL((k_amp_fused<2, true>), grid, block, lds, s, t0, t1, 0, a, m.n,
                                  m.n_tiles, m.W, m.wpad, vp, m.d_partials, m.rec_len);
        else
            hipExtLaunchKernelGGL((k_amp_fused<2, false>), grid, block, lds, s, t0, t1, 0, a, m.n,
                                  m.n_tiles, m.W, m.wpad, vp, m.d_partials, m.rec_len);
    }
    return hipGetLastError();
}

// complex64 padded copy of the amplitudes (complex128 input rounded to nearest)
__global__ void k_pack_amp(const void* __restrict__ src, bool c128, int64_t n, int W, int wpad,
                           int64_t total, float2* __restrict__ dst)
{
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = g / wpad;
        const int a = (int)(g % wpad);
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

hipError_t launch_pack_amp(const void* src, bool src_c128, int64_t n, int W, int wpad,
                           int64_t n_pad, float* dst, hipStream_t s)
{
    const int64_t total = n_pad * wpad;
    int64_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_pack_amp, dim3((int)g), dim3(256), 0, s, src, src_c128, n, W, wpad,
                       total, (float2*)dst);
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
// (the derivative of Eq. 1).  Per block, tiles of 64 events:
//   1. the tile's amplitudes into LDS (coalesced 16-byte loads);
//   2. wavefront 0, lane = event: S_i and w_i = 1 / I_i in FP64;
//   3. all threads: J_i into LDS as a 64 x PJ array (PJ = 2W rounded up to 4);
//   4. thread t: the 4 x 4 blocks (bp, bq), bp <= bq, numbered t % npair, over
//      the events of its split t / npair (splits of the 64 events when fewer
//      than 256 pairs), 16 FP64 accumulators per block.
// Record per block: [n_bad, then 16 doubles per block pair].
constexpr int kHessThreads = 256;

__host__ __device__ inline int hess_pj(int W) { return (2 * W + 3) / 4 * 4; }
__host__ __device__ inline int hess_npair(int W)
{
    const int nb = hess_pj(W) / 4;
    return nb * (nb + 1) / 2;
}
__host__ __device__ inline int hess_rec_len(int W) { return 1 + 16 * hess_npair(W); }
__host__ __device__ inline size_t hess_lds_bytes(int wpad)
{
    const int W = wpad;   // upper bound of the wave count
    const size_t main = (size_t)kAmpTile * amp_lds_stride_words(wpad) * 4   // amplitude tile
                        + (size_t)kAmpTile * hess_pj(W) * 8                  // J
                        + (size_t)kAmpTile * 16 + (size_t)kAmpTile * 8       // S, w
                        + 16;                                                // n_bad
    const size_t combine = (size_t)kHessThreads * 16 * 8;   // partial blocks at the end
    return (main > combine ? main : combine) + 16;
}

__global__ __launch_bounds__(kHessThreads) void k_amp_hessian(const float4* __restrict__ amp,
                                                              int64_t n_events, int64_t n_tiles,
                                                              int W, int wpad, VParams vp,
                                                              double* __restrict__ recs)
{
    extern __shared__ double lds_d[];
    char* lds = reinterpret_cast<char*>(lds_d);
    const int stride = amp_lds_stride_words(wpad) * 4;
    const int PJ = hess_pj(W);
    const int nb = PJ / 4;
    const int npair = nb * (nb + 1) / 2;
    char* tile = lds;
    double* s_J = reinterpret_cast<double*>(tile + (size_t)kAmpTile * stride);
    double2* s_S = reinterpret_cast<double2*>(s_J + (size_t)kAmpTile * PJ);
    double* s_w = reinterpret_cast<double*>(s_S + kAmpTile);
    // the count sits past both the tile data and the combine area
    int* s_bad = reinterpret_cast<int*>(lds + hess_lds_bytes(wpad) - 16);
    const int h = wpad >> 1;
    const int tid = threadIdx.x;

    // this thread's block pairs and event split
    const int splits = npair >= kHessThreads ? 1 : kHessThreads / npair;
    const int split = tid / (npair < kHessThreads ? npair : kHessThreads);
    const int pair0 = tid % (npair < kHessThreads ? npair : kHessThreads);
    const bool active = split < splits;
    constexpr int kMaxPairs = 3;   // pairs per thread: npair <= 3 * 256 (W <= 64)
    double acc[kMaxPairs][16];
    int bp[kMaxPairs], bq[kMaxPairs];
#pragma unroll
    for (int r = 0; r < kMaxPairs; ++r) {
        const int pr = pair0 + r * kHessThreads;
        bp[r] = bq[r] = -1;
        if (active && (r == 0 || npair > kHessThreads) && pr < npair) {
            // pair index -> (bp, bq), row-major upper triangle
            int rem = pr, row = 0;
            while (rem >= nb - row) {
                rem -= nb - row;
                ++row;
            }
            bp[r] = row;
            bq[r] = row + rem;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[r][k] = 0.0;
    }
    if (tid == 0) *s_bad = 0;

    const int64_t t0 = (int64_t)blockIdx.x * n_tiles / gridDim.x;
    const int64_t t1 = (int64_t)(blockIdx.x + 1) * n_tiles / gridDim.x;
    for (int64_t t = t0; t < t1; ++t) {
        const float4* src = amp + t * kAmpTile * h;
        for (int f = tid; f < kAmpTile * h; f += blockDim.x) {
            const int ev = f / h, c = f - ev * h;
            *reinterpret_cast<float4*>(tile + ev * stride + c * 16) = src[f];
        }
        __syncthreads();
        if (tid < kAmpTile) {
            const char* row = tile + tid * stride;
            double sr = 0.0, si = 0.0;
            for (int a = 0; a < W; ++a) {
                const float2 x = *reinterpret_cast<const float2*>(row + a * 8);
                const double vr = vp.v[2 * a], vi = vp.v[2 * a + 1];
                sr += vr * (double)x.x - vi * (double)x.y;
                si += vr * (double)x.y + vi * (double)x.x;
            }
            const double I = sr * sr + si * si;
            const bool valid = t * kAmpTile + tid < n_events;
            const bool ok = valid && (I > 0.0) && (I < INFINITY);
            if (valid && !ok) atomicAdd(s_bad, 1);   // LDS count, order-free
            s_S[tid] = make_double2(sr, si);
            // NaN for a degenerate event (its J, and so H, become NaN), 0 for padding
            s_w[tid] = ok ? 2.0 / I : (valid ? NAN : 0.0);
        }
        __syncthreads();
        for (int f = tid; f < kAmpTile * PJ; f += blockDim.x) {
            const int ev = f / PJ, p = f - ev * PJ;
            double j = 0.0;
            if (p < 2 * W) {
                const int b = p >> 1;
                const float2 x = *reinterpret_cast<const float2*>(tile + ev * stride + b * 8);
                const double2 S = s_S[ev];
                // z = conj(S) A_b
                const double zr = S.x * (double)x.x + S.y * (double)x.y;
                const double zi = S.x * (double)x.y - S.y * (double)x.x;
                j = s_w[ev] * ((p & 1) ? -zi : zr);
            }
            s_J[f] = j;
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int r = 0; r < kMaxPairs; ++r) {
                if (bp[r] < 0) continue;
                for (int ev = split; ev < kAmpTile; ev += splits) {
                    const double* Jr = s_J + ev * PJ;
                    const double2 a01 = *reinterpret_cast<const double2*>(Jr + 4 * bp[r]);
                    const double2 a23 = *reinterpret_cast<const double2*>(Jr + 4 * bp[r] + 2);
                    const double2 b01 = *reinterpret_cast<const double2*>(Jr + 4 * bq[r]);
                    const double2 b23 = *reinterpret_cast<const double2*>(Jr + 4 * bq[r] + 2);
                    const double ai[4] = {a01.x, a01.y, a23.x, a23.y};
                    const double bj[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) acc[r][4 * i + j] += ai[i] * bj[j];
                }
            }
        }
        __syncthreads();
    }

    // combine the event splits of each pair in split order, write the record
    double* rec = recs + (int64_t)blockIdx.x * hess_rec_len(W);
    double* s_part = reinterpret_cast<double*>(lds);   // reuses the tile area
    for (int r = 0; r < kMaxPairs; ++r) {
        if (r > 0 && npair <= kHessThreads) break;
        __syncthreads();
        if (active && bp[r] >= 0)
            for (int k = 0; k < 16; ++k) s_part[(size_t)tid * 16 + k] = acc[r][k];
        __syncthreads();
        const int base = r * kHessThreads;
        const int np_here = min(npair - base, kHessThreads);
        for (int e = tid; e < np_here * 16; e += blockDim.x) {
            const int pr = e / 16, k = e % 16;
            double x = 0.0;
            for (int sp = 0; sp < splits; ++sp) x += s_part[(size_t)(sp * npair + pr) * 16 + k];
            rec[1 + (size_t)(base + pr) * 16 + k] = x;
        }
    }
    if (tid == 0) rec[0] = (double)*s_bad;
}

// Sum of the block records in block order; one thread per entry of the
// 2W x 2W matrix (full, row-major), written to pinned host memory.
__global__ __launch_bounds__(256) void k_hess_assemble(const double* __restrict__ recs, int rows,
                                                       int W, double* out,
                                                       unsigned long long* done,
                                                       unsigned long long seq)
{
    const int P = 2 * W;
    const int rl = hess_rec_len(W);
    const int nb = hess_pj(W) / 4;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < P * P) {
        const int p = e / P, q = e % P;
        int i = p / 4, j = q / 4;
        int pp = p % 4, qq = q % 4;
        if (i > j) {   // the lower triangle mirrors the upper
            const int ti = i, tp = pp;
            i = j;
            pp = qq;
            j = ti;
            qq = tp;
        }
        const int pair = i * nb - i * (i - 1) / 2 + (j - i);
        const int col = 1 + pair * 16 + 4 * pp + qq;
        double x = 0.0, bad = 0.0;
        constexpr int kB = 16;
        for (int r0 = 0; r0 < rows; r0 += kB) {
            double v[kB], bv[kB];
#pragma unroll
            for (int k = 0; k < kB; ++k) {
                v[k] = r0 + k < rows ? recs[(int64_t)(r0 + k) * rl + col] : 0.0;
                bv[k] = r0 + k < rows ? recs[(int64_t)(r0 + k) * rl] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < kB; ++k) {
                x += v[k];
                bad += bv[k];
            }
        }
        store_system(out + e, bad > 0.0 ? NAN : x);
    }
    wait_vm_complete();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(done + blockIdx.x, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

int hess_grid(const Model& m) { return (int)std::min<int64_t>(2 * m.cus, std::max<int64_t>(1, m.n_tiles)); }
int hess_rows(const Model& m) { return hess_grid(m); }
int hess_rec_doubles(int W) { return hess_rec_len(W); }
int hess_assemble_blocks(int W) { return (4 * W * W + 255) / 256; }

hipError_t launch_hessian(const Model& m, const VParams& vp, double* recs, double* out,
                          unsigned long long* done, unsigned long long seq, hipStream_t s)
{
    const size_t lds = hess_lds_bytes(m.wpad);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void*)&k_amp_hessian,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_amp_hessian, dim3(hess_grid(m)), dim3(kHessThreads), lds, s,
                       (const float4*)m.d_data, m.n, m.n_tiles, m.W, m.wpad, vp, recs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hess_assemble, dim3(hess_assemble_blocks(m.W)), dim3(256), 0, s, recs,
                       hess_rows(m), m.W, out, done, seq);
    return hipGetLastError();
}

}  // namespace pwa
