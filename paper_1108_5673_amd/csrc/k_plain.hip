// k_plain.hip -- the plain double-precision table path: the straightforward
// implementation of Eq. 3 that the fused kernel is measured against.
//
// Table: complex128, packed entries (a <= a'), entry-major: T[e][i] for event i,
// so that one thread per event reads coalesced across a wavefront.
// Pass 1: one thread per event forms I_i = sum_e Re(c_e T_ie), writes
//         w_i = 1/I_i to memory and adds ln I_i to its block's partial.
// Pass 2: reads the whole table again: block (chunk, e) sums T_ie w_i over
//         the chunk's events, giving the per-chunk partial of U_e.
// No data reuse between the passes, no LDS staging of the table.
#include <hip/hip_runtime.h>

#include "pwa_internal.h"
#include "wave_ops.h"

namespace pwa {

constexpr int kPlainChunk = 4096;   // events per block of either pass

// x conj(y) with separately rounded products (no fused multiply-add)
__device__ inline double2 herm_product_soa(double xr, double xi, double yr, double yi)
{
#pragma clang fp contract(off)
    double2 t;
    t.x = xr * yr + xi * yi;
    t.y = xi * yr - xr * yi;
    return t;
}

__global__ void k_pack_soa(const void* __restrict__ src, bool src_is_table, bool src_c128,
                           int64_t n, int W, int P, const uint32_t* __restrict__ pairs,
                           double* __restrict__ dst)
{
    const int64_t total = n * P;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int e = (int)(g / n);
        const int64_t i = g % n;
        double2 t;
        if (src_is_table) {
            if (src_c128) t = reinterpret_cast<const double2*>(src)[i * P + e];
            else {
                const float2 f = reinterpret_cast<const float2*>(src)[i * P + e];
                t = make_double2(f.x, f.y);
            }
        } else {
            const uint32_t pr = pairs[e];
            const int a = (int)(pr & 0xffffu), b = (int)(pr >> 16);
            double xr, xi, yr, yi;
            if (src_c128) {
                const double2 x = reinterpret_cast<const double2*>(src)[i * W + a];
                const double2 y = reinterpret_cast<const double2*>(src)[i * W + b];
                xr = x.x; xi = x.y; yr = y.x; yi = y.y;
            } else {
                const float2 x = reinterpret_cast<const float2*>(src)[i * W + a];
                const float2 y = reinterpret_cast<const float2*>(src)[i * W + b];
                xr = x.x; xi = x.y; yr = y.x; yi = y.y;
            }
            t = herm_product_soa(xr, xi, yr, yi);
        }
        reinterpret_cast<double2*>(dst)[(int64_t)e * n + i] = t;
    }
}

__global__ void k_unpack_soa(const double* __restrict__ src, int64_t n, int P,
                             double* __restrict__ dst)
{
    const int64_t total = n * P;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = g / P;
        const int e = (int)(g % P);
        reinterpret_cast<double2*>(dst)[g] = reinterpret_cast<const double2*>(src)[(int64_t)e * n + i];
    }
}

static int grid_for(int64_t total, int block)
{
    int64_t g = (total + block - 1) / block;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_pack_soa(const void* src, bool src_is_table, bool src_c128, int64_t n, int W,
                           int P, const uint32_t* pairs, double* dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_soa, dim3(grid_for(n * P, 256)), dim3(256), 0, s, src,
                       src_is_table, src_c128, n, W, P, pairs, dst);
    return hipGetLastError();
}

hipError_t launch_unpack_soa(const double* src, int64_t n, int P, double* dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_unpack_soa, dim3(grid_for(n * P, 256)), dim3(256), 0, s, src, n, P,
                       dst);
    return hipGetLastError();
}

// Fixed-order block sum through LDS (blockDim.x == 256).
__device__ inline double block_sum(double x, double* sh)
{
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
        if ((int)threadIdx.x < m) sh[threadIdx.x] += sh[threadIdx.x + m];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_plain_intensity(const double2* __restrict__ T,
                                                         int64_t n, int P,
                                                         const uint32_t* __restrict__ pairs,
                                                         VParams vp, double* __restrict__ wout,
                                                         double* __restrict__ partials,
                                                         int rec_len)
{
    extern __shared__ double2 s_c[];     // P coefficients
    __shared__ double s_red[256];
    for (int e = threadIdx.x; e < P; e += blockDim.x) {
        const uint32_t pr = pairs[e];
        const int a = (int)(pr & 0xffffu), b = (int)(pr >> 16);
        const double* v = vsrc(vp);
        const double vr = v[2 * a], vi = v[2 * a + 1];
        const double wr = v[2 * b], wi = v[2 * b + 1];
        const double f = (a == b) ? 1.0 : 2.0;
        s_c[e] = make_double2(f * (vr * wr + vi * wi), f * (vi * wr - vr * wi));
    }
    __syncthreads();
    double dsum = 0.0, nbad = 0.0;
    const int64_t i0 = (int64_t)blockIdx.x * kPlainChunk;
    for (int r = 0; r < kPlainChunk / 256; ++r) {
        const int64_t i = i0 + r * 256 + threadIdx.x;
        if (i >= n) break;
        double I = 0.0;
        for (int e = 0; e < P; ++e) {
            const double2 t = T[(int64_t)e * n + i];
            const double2 c = s_c[e];
            I += c.x * t.x - c.y * t.y;
        }
        const bool ok = (I > 0.0) && (I < INFINITY);
        if (ok) dsum += log(I);
        else nbad += 1.0;
        wout[i] = ok ? 1.0 / I : NAN;   // a degenerate event makes the gradient NaN
    }
    dsum = block_sum(dsum, s_red);
    nbad = block_sum(nbad, s_red);
    if (threadIdx.x == 0) {
        partials[(int64_t)blockIdx.x * rec_len + 0] = dsum;
        partials[(int64_t)blockIdx.x * rec_len + 1] = nbad;
    }
}

__global__ __launch_bounds__(256) void k_plain_adjoint(const double2* __restrict__ T, int64_t n,
                                                       const double* __restrict__ w,
                                                       double* __restrict__ partials,
                                                       int rec_len)
{
    __shared__ double s_red[256];
    const int e = blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.x * kPlainChunk;
    double sr = 0.0, si = 0.0;
    for (int r = 0; r < kPlainChunk / 256; ++r) {
        const int64_t i = i0 + r * 256 + threadIdx.x;
        if (i >= n) break;
        const double2 t = T[(int64_t)e * n + i];
        const double wi = w[i];
        sr += t.x * wi;
        si += t.y * wi;
    }
    sr = block_sum(sr, s_red);
    si = block_sum(si, s_red);
    if (threadIdx.x == 0) {
        partials[(int64_t)blockIdx.x * rec_len + 2 + 2 * e] = sr;
        partials[(int64_t)blockIdx.x * rec_len + 3 + 2 * e] = si;
    }
}

int plain_rows(int64_t n) { return (int)((n + kPlainChunk - 1) / kPlainChunk); }

hipError_t launch_plain(const Model& m, const VParams& vp, bool grad, hipStream_t s,
                        const LaunchEvents& ev)
{
    const int rows = plain_rows(m.n);
    // timed from the start of the first pass to the end of the last one
    hipExtLaunchKernelGGL(k_plain_intensity, dim3(rows), dim3(256), sizeof(double2) * m.P, s,
                          ev.start, grad ? nullptr : ev.stop, 0, (const double2*)m.d_data, m.n,
                          m.P, m.d_pairs, vp, m.d_w, m.d_partials, m.rec_len);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess || !grad) return err;
    hipExtLaunchKernelGGL(k_plain_adjoint, dim3(rows, m.P), dim3(256), 0, s, nullptr, ev.stop, 0,
                          (const double2*)m.d_data, m.n, m.d_w, m.d_partials, m.rec_len);
    return hipGetLastError();
}

}  // namespace pwa
