// k_table.hip -- the per-event lookup table of Sec. 2 (T_i,aa' = A_a A*_a',
// precomputed because masses and widths are fixed) and the fused one-pass
// NLL + gradient kernel that streams it on every fit iteration (Eq. 3).
//
// Stored entries.  T_i is Hermitian, so only the upper triangle is kept and
// its real diagonal is stored in pairs of real values (see kDiagPair in
// pwa_internal.h): ps = ceil(W/2) + W(W-1)/2 complex entries per event (200
// at W = 20, 1600 bytes per event in complex64).
//
// Tiled layout (chosen for the streaming kernel).  A tile holds kTileEvents
// consecutive events.  Its ps stored entries are cut into slots of 64
// entries: slot k holds entries 64k .. 64k + n_k - 1, n_k = min(64, ps - 64k).
// Inside a slot the 16-byte vectors are ordered [vector v][lane], lane = e mod
// 64, and one vector holds EV = 16 / esz consecutive events of one entry (EV =
// 2 for complex64, 1 for complex128).  One wavefront load instruction
// therefore reads 64 x 16 = 1024 contiguous bytes (n_k x 16 in the last
// slot), lane l always receives entry 64k + l, and a wave's tile is one
// contiguous block of ps * kTileEvents * esz bytes.  The table is not padded
// in the entry direction; only the last tile is padded with zero events.
#include <hip/hip_runtime.h>

#include "pwa_internal.h"
#include "wave_ops.h"

namespace pwa {

__host__ __device__ inline int64_t tiled_offset(int64_t i, int e, int P, int esz)
{
    const int64_t t = i / kTileEvents;
    const int j = (int)(i % kTileEvents);
    const int ev = 16 / esz;
    const int k = e >> 6, lane = e & 63;
    const int nk = (P - 64 * k) < 64 ? (P - 64 * k) : 64;
    return t * (int64_t)P * kTileEvents * esz + (int64_t)k * 64 * kTileEvents * esz +
           (int64_t)((j / ev) * nk + lane) * 16 + (j % ev) * esz;
}

// T = x conj(y) in FP64 with each product rounded separately (no fused
// multiply-add), so that the table repeats a plain FP64 evaluation bit for bit.
__device__ inline double2 herm_product(double xr, double xi, double yr, double yi)
{
#pragma clang fp contract(off)
    double2 t;
    t.x = xr * yr + xi * yi;
    t.y = xi * yr - xr * yi;
    return t;
}

__device__ inline double2 load_c(const void* p, int64_t idx, bool c128)
{
    if (c128) return reinterpret_cast<const double2*>(p)[idx];
    const float2 f = reinterpret_cast<const float2*>(p)[idx];
    return make_double2((double)f.x, (double)f.y);
}

// One thread per stored 16-byte vector (the EV events of one entry that share
// it), one tile per block at a time: the lanes of a wavefront write the
// consecutive vectors of one (slot, vector) pair, so a wavefront stores up to
// 1 KB contiguous (non-temporal: the table is not read back by this kernel).
// From amplitudes, the tile's 16 events are first staged in LDS in FP64; the
// entry descriptors are kept in LDS.  Off the diagonal an entry is
// T_ab = A_a conj(A_b); a diagonal pair holds (|A_a|^2, |A_a2|^2), each formed
// exactly as the real part of the same product.  From a canonical packed
// table, the entries are copied (a diagonal pair takes the real parts of
// T_aa and T_a2a2).
constexpr int kPackMaxW = PWA_MAX_WAVES_TABLE;
__global__ __launch_bounds__(256) void k_pack_tiled(const void* __restrict__ src,
                                                    bool src_is_table, bool src_c128, int64_t n,
                                                    int W, int ps,
                                                    const uint32_t* __restrict__ slots,
                                                    bool store_c128, int64_t n_tiles,
                                                    void* __restrict__ dst)
{
    __shared__ double2 s_a[kTileEvents * kPackMaxW];
    __shared__ uint32_t s_desc[kPackMaxW / 2 + kPackMaxW * (kPackMaxW - 1) / 2];
    const int ev = store_c128 ? 1 : 2;           // events per vector
    const int nvec = kTileEvents / ev;           // vectors per entry and tile
    const int per_tile = ps * nvec;              // vectors per tile
    const int nslot = (ps + 63) / 64;            // slots of 64 entries
    const int P = W * (W + 1) / 2;               // canonical entries of a source table
    for (int e = threadIdx.x; e < ps; e += blockDim.x) s_desc[e] = slots[e];
    __syncthreads();
    // entry e of event j of the tile (zero for padding events)
    auto entry = [&](int64_t ibase, int j, int e) -> double2 {
        const uint32_t d = s_desc[e];
        const int a = (int)(d & 0xffffu), b = (int)((d >> 16) & kNoWave);
        if (src_is_table) {
            const int64_t i = ibase + j;
            if (i >= n) return make_double2(0.0, 0.0);
            if (d & kDiagPair)
                return make_double2(load_c(src, i * P + packed_index(W, a, a), src_c128).x,
                                    b < W ? load_c(src, i * P + packed_index(W, b, b), src_c128).x
                                          : 0.0);
            return load_c(src, i * P + packed_index(W, a, b), src_c128);
        }
        const double2 x = s_a[j * W + a];
        if (d & kDiagPair) {
            double im = 0.0;
            if (b < W) {
                const double2 y = s_a[j * W + b];
                im = herm_product(y.x, y.y, y.x, y.y).x;
            }
            return make_double2(herm_product(x.x, x.y, x.x, x.y).x, im);
        }
        const double2 y = s_a[j * W + b];
        return herm_product(x.x, x.y, y.x, y.y);
    };
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int64_t ibase = t * kTileEvents;
        if (!src_is_table) {
            __syncthreads();   // the previous tile's reads are done
            for (int x = threadIdx.x; x < kTileEvents * W; x += blockDim.x) {
                const int64_t i = ibase + x / W;
                s_a[x] = i < n ? load_c(src, ibase * W + x, src_c128) : make_double2(0.0, 0.0);
            }
            __syncthreads();
        }
        char* tb = reinterpret_cast<char*>(dst) + t * (int64_t)per_tile * 16;
        // wavefront w takes the (slot, vector) pairs w, w + 4, ... of the tile,
        // lane l entry 64 slot + l of it (the slot's nk entries are nk
        // consecutive vectors): the index arithmetic is per wavefront
        const int lane = threadIdx.x & 63;
        const int nwave = blockDim.x >> 6;
        for (int kv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); kv < nslot * nvec;
             kv += nwave) {
            const int k = kv / nvec, v = kv - k * nvec;   // slot, vector
            const int nk = (ps - 64 * k) < 64 ? (ps - 64 * k) : 64;
            if (lane >= nk) continue;
            const int o = k * 64 * nvec + v * nk + lane;
            const int e = 64 * k + lane;
            const int j0 = v * ev;               // first event of the vector in the tile
            const double2 t0 = entry(ibase, j0, e);
            const double2 t1 = ev == 2 ? entry(ibase, j0 + 1, e) : make_double2(0.0, 0.0);
            if (store_c128) {
                typedef double d2v __attribute__((ext_vector_type(2)));
                d2v q = {t0.x, t0.y};
                __builtin_nontemporal_store(q, reinterpret_cast<d2v*>(tb + (int64_t)o * 16));
            } else {
                typedef float f4v __attribute__((ext_vector_type(4)));
                f4v q = {(float)t0.x, (float)t0.y, (float)t1.x, (float)t1.y};
                __builtin_nontemporal_store(q, reinterpret_cast<f4v*>(tb + (int64_t)o * 16));
            }
        }
    }
}

// Diagonal entries of a canonical packed source table whose imaginary part is
// not zero (or not a number): a Hermitian table has none.
__global__ void k_check_table_diag(const void* __restrict__ src, bool c128, int64_t n, int W,
                                   unsigned long long* __restrict__ count)
{
    const int P = W * (W + 1) / 2;
    const int64_t total = n * W;
    unsigned long long bad = 0;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = g / W;
        const int a = (int)(g % W);
        const double im = load_c(src, i * P + packed_index(W, a, a), c128).y;
        if (!(im == 0.0)) ++bad;
    }
    bad = (unsigned long long)wave_allsum_int((int)bad);
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd(count, bad);
}

// The canonical packed table (N x P, complex, entries a <= b in row-major
// order) from the tiled store; a diagonal entry comes back with a zero
// imaginary part.
__global__ void k_unpack_tiled(const void* __restrict__ src, bool c128, int64_t n, int W,
                               const uint32_t* __restrict__ pairs, void* __restrict__ dst)
{
    const int esz = c128 ? 16 : 8;
    const int P = W * (W + 1) / 2;
    const int ps = tiled_entries(W);
    const int64_t total = n * P;
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = g / P;
        const uint32_t pr = pairs[g % P];
        const int a = (int)(pr & 0xffffu), b = (int)(pr >> 16);
        const int se = a == b ? a / 2 : tiled_offdiag_index(W, a, b);
        const char* s = reinterpret_cast<const char*>(src) + tiled_offset(i, se, ps, esz);
        double2 x = load_c(s, 0, c128);
        if (a == b) x = make_double2((a & 1) ? x.y : x.x, 0.0);
        if (c128) reinterpret_cast<double2*>(dst)[g] = x;
        else reinterpret_cast<float2*>(dst)[g] = make_float2((float)x.x, (float)x.y);
    }
}

static int grid_for(int64_t total, int block)
{
    int64_t g = (total + block - 1) / block;
    if (g > 65536) g = 65536;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_pack_tiled(const void* src, bool src_is_table, bool src_c128, int64_t n,
                             int W, int ps, const uint32_t* slots, bool store_c128,
                             int64_t n_tiles, void* dst, hipStream_t s, const LaunchEvents& ev)
{
    const int64_t g = n_tiles < 4096 ? (n_tiles < 1 ? 1 : n_tiles) : 4096;
    hipExtLaunchKernelGGL(k_pack_tiled, dim3((int)g), dim3(256), 0, s, ev.start, ev.stop, 0, src,
                          src_is_table, src_c128, n, W, ps, slots, store_c128, n_tiles, dst);
    return hipGetLastError();
}

hipError_t launch_check_table_diag(const void* src, bool c128, int64_t n, int W,
                                   unsigned long long* count, hipStream_t s)
{
    hipLaunchKernelGGL(k_check_table_diag, dim3(grid_for(n * W, 256)), dim3(256), 0, s, src, c128,
                       n, W, count);
    return hipGetLastError();
}

// Reference reader: streams n_vec 16-byte vectors once with the same
// non-temporal loads and the same shape as the fused kernel (one 1024-thread
// block per compute unit, a contiguous range per block, 1 KB per wavefront
// load), with up to twelve loads per lane in flight and no arithmetic on the data
// beyond an xor that keeps the loads alive.  It measures the read bandwidth
// the streaming kernels can reach on the same bytes.  Each block stores one
// word, and only if its xor is the (practically impossible) value `magic`.
constexpr int kReadUnroll = 6;
typedef float rd4 __attribute__((ext_vector_type(4)));

__device__ __attribute__((always_inline)) inline void read_round(rd4 (&r)[kReadUnroll],
                                                                  const float4* p, int64_t v0,
                                                                  int64_t v1, int64_t c, int nw,
                                                                  int lane)
{
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u) {
        const int64_t idx = v0 + 64 * (c + (int64_t)u * nw) + lane;
        r[u] = idx < v1 ? __builtin_nontemporal_load(reinterpret_cast<const rd4*>(p + idx))
                        : rd4{0.f, 0.f, 0.f, 0.f};
    }
}

__device__ __attribute__((always_inline)) inline uint32_t fold_round(const rd4 (&r)[kReadUnroll])
{
    uint32_t a = 0;
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u)
        a ^= __float_as_uint(r[u].x) ^ __float_as_uint(r[u].y) ^ __float_as_uint(r[u].z) ^
             __float_as_uint(r[u].w);
    return a;
}

__global__ __launch_bounds__(1024) void k_stream_read(const float4* __restrict__ p, int64_t n_vec,
                                                      uint32_t magic, uint32_t* __restrict__ sink)
{
    const int64_t v0 = (int64_t)blockIdx.x * n_vec / gridDim.x;
    const int64_t v1 = (int64_t)(blockIdx.x + 1) * n_vec / gridDim.x;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t acc = 0;
    // 64-vector chunks of the range: wavefront w takes chunks w, w + nw, ...,
    // kReadUnroll of them per round; the next round's loads are issued before
    // this round's values are used (two register buffers)
    const int64_t step = (int64_t)nw * kReadUnroll;
    rd4 x[kReadUnroll], y[kReadUnroll];
    int64_t c = wave;
    if (v0 + 64 * c < v1) read_round(x, p, v0, v1, c, nw, lane);
    for (; v0 + 64 * c < v1; c += 2 * step) {
        const bool more = v0 + 64 * (c + step) < v1;
        if (more) read_round(y, p, v0, v1, c + step, nw, lane);
        acc ^= fold_round(x);
        if (!more) break;
        if (v0 + 64 * (c + 2 * step) < v1) read_round(x, p, v0, v1, c + 2 * step, nw, lane);
        acc ^= fold_round(y);
    }
    if (acc == magic) sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

hipError_t launch_stream_read(const void* p, int64_t bytes, uint32_t* sink, int sink_len,
                              hipStream_t s, const LaunchEvents& ev)
{
    const int64_t n_vec = bytes / 16;
    hipExtLaunchKernelGGL(k_stream_read, dim3(sink_len / 1024), dim3(1024), 0, s, ev.start,
                          ev.stop, 0, (const float4*)p, n_vec, 0x9e3779b9u, sink);
    return hipGetLastError();
}

hipError_t launch_unpack_tiled(const void* src, bool c128, int64_t n, int W,
                               const uint32_t* pairs, void* dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_unpack_tiled, dim3(grid_for(n * (W * (W + 1) / 2), 256)), dim3(256), 0,
                       s, src, c128, n, W, pairs, dst);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused one-pass NLL + gradient over the tiled table.
//
// A wavefront works on E events at a time (a sub-tile).  Lane l owns entries
// e = 64k + l (k < K) for the whole kernel:
//   1. loads its entries of the E events (dwordx4, 1 KB per instruction);
//   2. forms its partial intensities p_j = sum_k Re(c_e T_je) in FP64, with
//      c_aa = |V_a|^2 and c_aa' = 2 V_a V*_a' (a < a'), so that
//      sum_e Re(c_e T_ie) = sum_a sum_a' V_a V*_a' T_i,aa' (Eq. 3, first bracket);
//   3. reduces the E partials over the 64 lanes with one transposing
//      butterfly (transpose_reduce), after which each run of 64/E lanes holds
//      the full I_i of one event;
//   4. forms w_i = 1/I_i in FP64 (invalid or padded events give 0) and
//      queues I_i for a batched ln (FusedState);
//   5. broadcasts w_i through scalar registers and accumulates, from the
//      registers loaded in step 1, U_e += w_i T_ie (FP64), the data part of
//      the gradient; the table is read from memory exactly once.
// At the end the wavefronts of a block are combined in LDS in a fixed order,
// the block contracts its U with V, u_b = sum_a V_a U_ab (U_ab = conj(U_ba),
// the diagonal from the stored pairs), and writes one partial record
// [sum ln I, n_bad, u_0, ..., u_{W-1}] (2 + 2W doubles).
// ---------------------------------------------------------------------------
template <typename S> struct Vec16;
template <> struct Vec16<float> {
    using T = float4;
    static constexpr int EV = 2;
    __device__ static T zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ static double re(const T& x, int h) { return h == 0 ? (double)x.x : (double)x.z; }
    __device__ static double im(const T& x, int h) { return h == 0 ? (double)x.y : (double)x.w; }
    __device__ static void opaque(T& x) { asm volatile("" : "+v"(x.x), "+v"(x.y), "+v"(x.z), "+v"(x.w)); }
    __device__ static T load(const char* p)
    {
        typedef float f4v __attribute__((ext_vector_type(4)));
        const f4v t = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
        return make_float4(t.x, t.y, t.z, t.w);
    }
};
template <> struct Vec16<double> {
    using T = double2;
    static constexpr int EV = 1;
    __device__ static T zero() { return make_double2(0.0, 0.0); }
    __device__ static double re(const T& x, int) { return x.x; }
    __device__ static double im(const T& x, int) { return x.y; }
    __device__ static void opaque(T&) {}
    __device__ static T load(const char* p)
    {
        typedef double d2v __attribute__((ext_vector_type(2)));
        const d2v t = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
        return make_double2(t.x, t.y);
    }
};

// One sub-tile's loaded vectors: lane l holds, for each slot k, the E events
// of entry 64k + l as E / EV 16-byte vectors.
template <typename S, int K, int E>
struct SubTile {
    using VT = Vec16<S>;
    using V4 = typename VT::T;
    static constexpr int EV = VT::EV;
    static constexpr int VS = E / EV;
    static constexpr int VPT = kTileEvents / EV;
    V4 x[K][VS];

    // tb is wave-uniform, so every address is a scalar base plus the lane's
    // 16-byte offset.  Full slots load unconditionally; only the last,
    // partly filled slot is predicated on the lane.  The table is read once
    // per evaluation, so the loads are non-temporal.
    //
    // From 8 slots on, every load is issued without a branch (written with
    // run-time slot tests, the compiler turned the wide shapes' loads into
    // one branch per slot that waited for its load, so that one load at a
    // time was in flight): a lane whose entry lies past the P stored entries
    // reads the last stored entry instead.  Its coefficient is zero, so it
    // adds nothing to I, and the U entry it feeds is never read.
    __device__ void load(const char* tb, int sub, int P, int lane)
    {
        if constexpr (K >= 8) {
            const int kl = (P - 1) >> 6;   // last slot holding entries
            const int nl = P - 64 * kl;    // entries in it
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int kk = k < kl ? k : kl;
                const int nk = k < kl ? 64 : nl;
                const int ln = k < kl ? lane : (k == kl ? min(lane, nl - 1) : nl - 1);
                const char* sb = tb + (int64_t)kk * 64 * VPT * 16;
#pragma unroll
                for (int v = 0; v < VS; ++v)
                    x[k][v] = VT::load(sb + ((sub * VS + v) * nk + ln) * 16);
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const char* sb = tb + (int64_t)k * 64 * VPT * 16;
            if (64 * (k + 1) <= P) {
#pragma unroll
                for (int v = 0; v < VS; ++v)
                    x[k][v] = VT::load(sb + ((sub * VS + v) * 64 + lane) * 16);
            } else if (64 * k < P) {
                const int nk = P - 64 * k;
#pragma unroll
                for (int v = 0; v < VS; ++v)
                    x[k][v] = lane < nk
                                  ? VT::load(sb + ((sub * VS + v) * nk + lane) * 16)
                                  : VT::zero();
            } else {
#pragma unroll
                for (int v = 0; v < VS; ++v) x[k][v] = VT::zero();
            }
        }
    }
};

// Per-lane running state.  ln I is not taken per sub-tile: after each
// sub-tile one lane of every run keeps its event's intensity in `held` (lane
// l % RUN == u % RUN), so that after RUN sub-tiles the 64 lanes hold 64
// different events and one logarithm per lane covers them all.
struct FusedState {
    double dsum;     // sum of ln I over this lane's flushed events
    double held;     // intensity waiting for its logarithm (1 when none)
    int nbad;        // invalid intensities seen by this lane (run leaders only)
};

// Steps 2-5 for one loaded sub-tile.
template <typename S, int K, int E, bool GRAD>
__device__ inline void process_subtile(SubTile<S, K, E>& st, const double2* s_c, int lane,
                                       int64_t u, int64_t first_event, int64_t n_events,
                                       double (&ur)[K], double (&ui)[K], FusedState& fs)
{
    using VT = Vec16<S>;
    constexpr int EV = VT::EV;
    constexpr int VS = E / EV;
    constexpr int RUN = 64 / E;
    double p[E];
#pragma unroll
    for (int j = 0; j < E; ++j) p[j] = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const double2 c = s_c[k * 64 + lane];
#pragma unroll
        for (int v = 0; v < VS; ++v)
#pragma unroll
            for (int h = 0; h < EV; ++h) {
                double& pj = p[v * EV + h];
                pj = __fma_rn(c.x, VT::re(st.x[k][v], h), pj);
                pj = __fma_rn(-c.y, VT::im(st.x[k][v], h), pj);
            }
    }
    // Keep the compiler from carrying FP64 copies of the loaded values from
    // step 2 to step 5 (that would double the register footprint); step 5
    // converts again from the loaded registers.
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int v = 0; v < VS; ++v) VT::opaque(st.x[k][v]);
    const double I = transpose_reduce<E>(p, lane);
    const int64_t evt = first_event + lane / RUN;
    const bool valid = evt < n_events;
    const bool ok = valid && (I > 0.0) && (I < INFINITY);
    // a degenerate event's weight is NaN, so that every gradient entry it
    // reaches is NaN; padding events weigh nothing
    const double w = ok ? recip_f64(I) : (valid ? NAN : 0.0);
    if ((lane % RUN) == 0 && valid && !ok) ++fs.nbad;
    if ((lane % RUN) == (int)(u % RUN) && ok) fs.held = I;
    if ((int)(u % RUN) == RUN - 1) {
        fs.dsum += log(fs.held);
        fs.held = 1.0;
    }
    if (GRAD) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const double wj = readlane_f64(w, j * RUN);
            const int v = j / EV, h = j % EV;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                ur[k] = __fma_rn(wj, VT::re(st.x[k][v], h), ur[k]);
                ui[k] = __fma_rn(wj, VT::im(st.x[k][v], h), ui[k]);
            }
        }
    }
}

// Block shape.  The shapes whose streaming loop fits in 128 registers (the
// 20-wave shapes) run one block of sixteen wavefronts per CU, four per SIMD,
// which also makes the per-block partial records few; the others run blocks
// of four wavefronts.
template <typename S, int K, int E>
constexpr int fused_threads()
{
    if constexpr (sizeof(S) == 4) return (K == 4 && E == 4) ? 1024 : 256;
    else return (K == 2 && E == 4) ? 1024 : 256;
}

// U_ab of the block's U (stored entries in LDS): off the diagonal the stored
// entry or its conjugate, on it one part of a stored pair.
__device__ inline double2 u_entry(const double2* s_ue, int W, int a, int b)
{
    if (a == b) {
        const double2 x = s_ue[a >> 1];
        return make_double2((a & 1) ? x.y : x.x, 0.0);
    }
    if (a < b) return s_ue[tiled_offdiag_index(W, a, b)];
    const double2 x = s_ue[tiled_offdiag_index(W, b, a)];
    return make_double2(x.x, -x.y);
}

// u_b = sum_a V_a U_ab for b < W from U in LDS, written to rec[2 + 2b]:
// thread t takes b = t / 32 (and b + blockDim / 32, ...) and the waves
// a = t % 32 + 32 m; the 32 partial sums of b are added by a fixed butterfly.
__device__ inline void contract_u(const double2* s_ue, const double* s_v, int W,
                                  double* __restrict__ rec)
{
    const int j = threadIdx.x & 31;
    for (int b0 = 0; b0 < W; b0 += blockDim.x >> 5) {
        const int b = b0 + (threadIdx.x >> 5);   // uniform over each half wavefront
        double xr = 0.0, xi = 0.0;
        if (b < W) {
            for (int a = j; a < W; a += 32) {
                const double2 u = u_entry(s_ue, W, a, b);
                const double vr = s_v[2 * a], vi = s_v[2 * a + 1];
                xr = __fma_rn(vr, u.x, __fma_rn(-vi, u.y, xr));
                xi = __fma_rn(vr, u.y, __fma_rn(vi, u.x, xi));
            }
        }
#pragma unroll
        for (int m = 16; m >= 1; m >>= 1) {
            xr += __shfl_xor(xr, m);
            xi += __shfl_xor(xi, m);
        }
        if (b < W && j == 0) *reinterpret_cast<double2*>(rec + 2 + 2 * b) = make_double2(xr, xi);
    }
}

template <typename S, int K, int E, bool GRAD>
__global__ __launch_bounds__((fused_threads<S, K, E>())) void k_table_fused(
    const char* __restrict__ table, int64_t n_events, int64_t n_tiles, int P, int W,
    const uint32_t* __restrict__ slots, VParams vp, double* __restrict__ partials, int rec_len)
{
    using VT = Vec16<S>;
    constexpr int esz = 2 * sizeof(S);
    constexpr int NSUB = kTileEvents / E;
    static_assert(E % VT::EV == 0 && kTileEvents % E == 0, "sub-tile shape");

    constexpr int NW = fused_threads<S, K, E>() / 64;
    constexpr bool kTree = (NW / 2 + 1) * K * 64 * 16 <= 65536;
    __shared__ double2 s_c[K * 64];
    __shared__ double2 s_u[GRAD ? (kTree ? NW / 2 : 1) * K * 64 : 1];
    __shared__ double s_misc[2 * NW];
    __shared__ double s_v[GRAD ? 2 * PWA_MAX_WAVES_TABLE : 1];

    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int nwaves = blockDim.x >> 6;

    // This wave's sub-tiles, in order: sub-tiles s0 + wave, s0 + wave + nwaves,
    // ... of the block's range (sub-tile s is part s % NSUB of tile s / NSUB;
    // sub-tiles rather than tiles are dealt out, so that the wavefronts'
    // shares differ by at most one sub-tile).  The next sub-tile is loaded
    // while the current one is processed (two register buffers); the first
    // load is issued before the coefficients are formed.
    const int64_t n_sub = n_tiles * NSUB;
    const int64_t s0 = (int64_t)blockIdx.x * n_sub / gridDim.x;
    const int64_t s1 = (int64_t)(blockIdx.x + 1) * n_sub / gridDim.x;
    const int64_t tile_bytes = (int64_t)P * kTileEvents * esz;
    const int64_t U = (s1 - s0 > wave) ? (s1 - s0 - wave + nwaves - 1) / nwaves : 0;
    auto sub_of = [&](int64_t u) { return s0 + wave + nwaves * u; };
    auto base_of = [&](int64_t u) { return table + (sub_of(u) / NSUB) * tile_bytes; };
    auto part_of = [&](int64_t u) { return (int)(sub_of(u) % NSUB); };
    auto first_of = [&](int64_t u) { return sub_of(u) * E; };

    SubTile<S, K, E> a, b;
    if (U > 0) a.load(base_of(0), part_of(0), P, lane);

    // coefficients c_e for every (slot, lane): 2 V_a V*_b off the diagonal,
    // |V_a|^2 - i |V_a2|^2 for a diagonal pair (so that Re(c_e T_ie) is the
    // entry's share of I_i in both cases)
    const double* v = vsrc(vp);
    for (int idx = threadIdx.x; idx < K * 64; idx += blockDim.x) {
        double2 c = make_double2(0.0, 0.0);
        if (idx < P) {
            const uint32_t d = slots[idx];
            const int wa = (int)(d & 0xffffu), wb = (int)((d >> 16) & kNoWave);
            const double vr = v[2 * wa], vi = v[2 * wa + 1];
            if (d & kDiagPair) {
                c.x = vr * vr + vi * vi;
                if (wb < W) c.y = -(v[2 * wb] * v[2 * wb] + v[2 * wb + 1] * v[2 * wb + 1]);
            } else {
                const double wr = v[2 * wb], wi = v[2 * wb + 1];
                c.x = 2.0 * (vr * wr + vi * wi);   // Re V_a V*_b
                c.y = 2.0 * (vi * wr - vr * wi);   // Im V_a V*_b
            }
        }
        s_c[idx] = c;
    }
    if (GRAD)
        for (int a = threadIdx.x; a < 2 * W; a += blockDim.x) s_v[a] = v[a];
    __syncthreads();

    double ur[K], ui[K];
#pragma unroll
    for (int k = 0; k < K; ++k) { ur[k] = 0.0; ui[k] = 0.0; }
    FusedState fs{0.0, 1.0, 0};

    if constexpr (K < 20) {
        for (int64_t u = 0; u < U; u += 2) {
            if (u + 1 < U) b.load(base_of(u + 1), part_of(u + 1), P, lane);
            process_subtile<S, K, E, GRAD>(a, s_c, lane, u, first_of(u), n_events, ur, ui, fs);
            if (u + 1 < U) {
                if (u + 2 < U) a.load(base_of(u + 2), part_of(u + 2), P, lane);
                process_subtile<S, K, E, GRAD>(b, s_c, lane, u + 1, first_of(u + 1), n_events, ur,
                                               ui, fs);
            }
        }
    } else {
        // 20 or more slots: one buffer (two, with the accumulators, take 400
        // or more registers from 24 slots and spill at 32); its loads are in
        // flight together
        for (int64_t u = 0; u < U; ++u) {
            if (u > 0) a.load(base_of(u), part_of(u), P, lane);
            process_subtile<S, K, E, GRAD>(a, s_c, lane, u, first_of(u), n_events, ur, ui, fs);
        }
    }

    // logarithms of the intensities still held, then the fixed-order combine
    // of the block's wavefronts
    fs.dsum += log(fs.held);
    const double dsum = wave_allsum(fs.dsum);
    const int nbad = wave_allsum_int(fs.nbad);
    if (lane == 0) {
        s_misc[2 * wave] = dsum;
        s_misc[2 * wave + 1] = (double)nbad;
    }
    double* rec = partials + (int64_t)blockIdx.x * rec_len;
    if (GRAD) {
        if constexpr (kTree) {
            // pairwise tree: at half-width h, wave w + h hands its sums to wave w
            for (int h = NW / 2; h >= 1; h >>= 1) {
                if (wave >= h && wave < 2 * h) {
#pragma unroll
                    for (int k = 0; k < K; ++k)
                        s_u[((wave - h) * K + k) * 64 + lane] = make_double2(ur[k], ui[k]);
                }
                __syncthreads();
                if (wave < h) {
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        const double2 o = s_u[(wave * K + k) * 64 + lane];
                        ur[k] += o.x;
                        ui[k] += o.y;
                    }
                }
                __syncthreads();
            }
            if (wave == 0) {
#pragma unroll
                for (int k = 0; k < K; ++k) s_u[k * 64 + lane] = make_double2(ur[k], ui[k]);
            }
            __syncthreads();
        } else {
            // one accumulator in LDS, the wavefronts adding in turn
            for (int w = 0; w < NW; ++w) {
                if (wave == w) {
#pragma unroll
                    for (int k = 0; k < K; ++k) {
                        double2 u = make_double2(ur[k], ui[k]);
                        if (w > 0) {
                            const double2 o = s_u[k * 64 + lane];
                            u.x += o.x;
                            u.y += o.y;
                        }
                        s_u[k * 64 + lane] = u;
                    }
                }
                __syncthreads();
            }
        }
        // s_u now holds the block's U over the stored entries
        contract_u(s_u, s_v, W, rec);
    } else {
        __syncthreads();
    }
    if (threadIdx.x < 2) {
        double x = 0.0;
        for (int w = 0; w < NW; ++w) x += s_misc[2 * w + threadIdx.x];
        rec[threadIdx.x] = x;
    }
}

// Instantiations: K slots of 64 entries per lane (P <= 64 K) and E events per
// sub-tile.  The default E keeps the loaded vectors near 64 registers; the
// other sub-tile widths are kept for tuning (PWA_TABLE_SUBTILE).
template <typename S, int K, int E>
static hipError_t run_fused(const Model& m, const VParams& vp, bool grad, hipStream_t s,
                            const LaunchEvents& ev)
{
    constexpr int NT = fused_threads<S, K, E>();
    if (grad)
        hipExtLaunchKernelGGL((k_table_fused<S, K, E, true>), dim3(m.grid), dim3(NT), 0, s,
                              ev.start, ev.stop, 0, (const char*)m.d_data, m.n, m.n_tiles, m.ps,
                              m.W, m.d_slots, vp, m.d_partials, m.rec_len);
    else
        hipExtLaunchKernelGGL((k_table_fused<S, K, E, false>), dim3(m.grid), dim3(NT), 0, s,
                              ev.start, ev.stop, 0, (const char*)m.d_data, m.n, m.n_tiles, m.ps,
                              m.W, m.d_slots, vp, m.d_partials, m.rec_len);
    return hipGetLastError();
}

// Reference reader of the tiled table: the fused kernel's loads (the same
// grid, block shape, sub-tile order and two register buffers) with all of its
// arithmetic taken out; an xor of the loaded bits keeps the loads alive, and
// a thread stores only if its xor is the (practically impossible) `magic`.
__device__ inline uint32_t bits_of(const float4& x)
{
    return __float_as_uint(x.x) ^ __float_as_uint(x.y) ^ __float_as_uint(x.z) ^
           __float_as_uint(x.w);
}
__device__ inline uint32_t bits_of(const double2& x)
{
    return (uint32_t)(__double2loint(x.x) ^ __double2hiint(x.x) ^ __double2loint(x.y) ^
                      __double2hiint(x.y));
}

template <typename S, int K, int E>
__device__ inline uint32_t fold_subtile(const SubTile<S, K, E>& st)
{
    uint32_t a = 0;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int v = 0; v < SubTile<S, K, E>::VS; ++v) a ^= bits_of(st.x[k][v]);
    return a;
}

template <typename S, int K, int E>
__global__ __launch_bounds__((fused_threads<S, K, E>())) void k_table_read(
    const char* __restrict__ table, int64_t n_tiles, int P, uint32_t magic,
    uint32_t* __restrict__ sink)
{
    constexpr int esz = 2 * sizeof(S);
    constexpr int NSUB = kTileEvents / E;
    const int lane = lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwaves = blockDim.x >> 6;
    const int64_t n_sub = n_tiles * NSUB;
    const int64_t s0 = (int64_t)blockIdx.x * n_sub / gridDim.x;
    const int64_t s1 = (int64_t)(blockIdx.x + 1) * n_sub / gridDim.x;
    const int64_t tile_bytes = (int64_t)P * kTileEvents * esz;
    const int64_t U = (s1 - s0 > wave) ? (s1 - s0 - wave + nwaves - 1) / nwaves : 0;
    auto sub_of = [&](int64_t u) { return s0 + wave + nwaves * u; };
    auto base_of = [&](int64_t u) { return table + (sub_of(u) / NSUB) * tile_bytes; };
    auto part_of = [&](int64_t u) { return (int)(sub_of(u) % NSUB); };
    SubTile<S, K, E> a, b;
    uint32_t acc = 0;
    if (U > 0) a.load(base_of(0), part_of(0), P, lane);
    for (int64_t u = 0; u < U; u += 2) {
        if (u + 1 < U) b.load(base_of(u + 1), part_of(u + 1), P, lane);
        acc ^= fold_subtile(a);
        if (u + 1 < U) {
            if (u + 2 < U) a.load(base_of(u + 2), part_of(u + 2), P, lane);
            acc ^= fold_subtile(b);
        }
    }
    if (acc == magic) sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

template <typename S, int K, int E>
static hipError_t run_read(const Model& m, uint32_t* sink, hipStream_t s, const LaunchEvents& ev)
{
    constexpr int NT = fused_threads<S, K, E>();
    hipExtLaunchKernelGGL((k_table_read<S, K, E>), dim3(m.grid), dim3(NT), 0, s, ev.start,
                          ev.stop, 0, (const char*)m.d_data, m.n_tiles, m.ps, 0x9e3779b9u, sink);
    return hipGetLastError();
}

template <typename S, int K, int E>
static const void* fused_fn()
{
    return (const void*)&k_table_fused<S, K, E, true>;
}

// Slots of 64 stored entries per lane: the fewest instantiated count that
// holds the P entries of an event.  From 8 on the counts step by 4 (every
// even count was measured and gave nothing more); 32 holds W <= 64.
int select_kslots(int P, bool c128)
{
    (void)c128;
    const int need = (P + 63) / 64;
    const int opts[] = {1, 2, 4, 8, 12, 16, 20, 24, 28, 32};
    for (int k : opts)
        if (k >= need) return k;
    return -1;
}

// Default sub-tile width per slot count: at most 8 loaded 16-byte vectors
// (32 registers) per lane and buffer, which with the second buffer of the
// software pipeline leaves room for three wavefronts per SIMD.
int default_subtile(int kslots, bool c128)
{
    int e = 8 / kslots * (c128 ? 1 : 2);
    if (e > kTileEvents) e = kTileEvents;
    if (e < (c128 ? 1 : 2)) e = c128 ? 1 : 2;
    return e;
}

// Calls f.template operator()<K, E>() for the instantiated (K, E) pair, or returns
// false when the pair is not instantiated.
template <typename S, typename F>
static bool with_shape(int K, int E, F&& f)
{
    constexpr bool F32 = sizeof(S) == 4;
#define PWA_SHAPE(k, e)                                \
    if (K == k && E == e) {                            \
        f.template operator()<k, e>();                 \
        return true;                                   \
    }
    if constexpr (F32) {
        PWA_SHAPE(1, 16)
        PWA_SHAPE(2, 8)
        PWA_SHAPE(4, 4)
        PWA_SHAPE(4, 8)
        PWA_SHAPE(8, 2)
        PWA_SHAPE(12, 2)
        PWA_SHAPE(16, 2)
        PWA_SHAPE(20, 2)
        PWA_SHAPE(24, 2)
        PWA_SHAPE(28, 2)
        PWA_SHAPE(32, 2)
    } else {
        PWA_SHAPE(1, 8)
        PWA_SHAPE(2, 4)
        PWA_SHAPE(4, 2)
        PWA_SHAPE(4, 4)
        PWA_SHAPE(8, 1)
        PWA_SHAPE(12, 1)
        PWA_SHAPE(16, 1)
        PWA_SHAPE(20, 1)
        PWA_SHAPE(24, 1)
        PWA_SHAPE(28, 1)
        PWA_SHAPE(32, 1)
    }
#undef PWA_SHAPE
    return false;
}

bool fused_shape_ok(const Model& m)
{
    bool ok = false;
    auto probe = [&]<int K, int E>() { ok = true; };
    if (m.form == kTable32) with_shape<float>(m.kslots, m.subtile, probe);
    else with_shape<double>(m.kslots, m.subtile, probe);
    return ok;
}

hipError_t launch_table_read(const Model& m, uint32_t* sink, hipStream_t s,
                             const LaunchEvents& ev)
{
    hipError_t err = hipErrorInvalidValue;
    if (m.form == kTable32) {
        auto go = [&]<int K, int E>() { err = run_read<float, K, E>(m, sink, s, ev); };
        with_shape<float>(m.kslots, m.subtile, go);
    } else {
        auto go = [&]<int K, int E>() { err = run_read<double, K, E>(m, sink, s, ev); };
        with_shape<double>(m.kslots, m.subtile, go);
    }
    return err;
}

int table_read_threads(const Model& m)
{
    int nt = 0;
    if (m.form == kTable32) {
        auto go = [&]<int K, int E>() { nt = fused_threads<float, K, E>(); };
        with_shape<float>(m.kslots, m.subtile, go);
    } else {
        auto go = [&]<int K, int E>() { nt = fused_threads<double, K, E>(); };
        with_shape<double>(m.kslots, m.subtile, go);
    }
    return nt;
}

hipError_t launch_table_fused(const Model& m, const VParams& vp, bool grad, hipStream_t s,
                              const LaunchEvents& ev)
{
    hipError_t err = hipErrorInvalidValue;
    if (m.form == kTable32) {
        auto go = [&]<int K, int E>() { err = run_fused<float, K, E>(m, vp, grad, s, ev); };
        with_shape<float>(m.kslots, m.subtile, go);
    } else {
        auto go = [&]<int K, int E>() { err = run_fused<double, K, E>(m, vp, grad, s, ev); };
        with_shape<double>(m.kslots, m.subtile, go);
    }
    return err;
}

int table_fused_grid(const Model& m)
{
    const void* fn = nullptr;
    int nt = 256;
    if (m.form == kTable32) {
        auto get = [&]<int K, int E>() {
            fn = fused_fn<float, K, E>();
            nt = fused_threads<float, K, E>();
        };
        with_shape<float>(m.kslots, m.subtile, get);
    } else {
        auto get = [&]<int K, int E>() {
            fn = fused_fn<double, K, E>();
            nt = fused_threads<double, K, E>();
        };
        with_shape<double>(m.kslots, m.subtile, get);
    }
    int per_cu = 0;
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nt, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int64_t g = (int64_t)m.cus * per_cu;
    const int64_t max_blocks = (m.n_tiles + nt / 64 - 1) / (nt / 64);
    if (g > max_blocks) g = max_blocks;
    return (int)(g < 1 ? 1 : g);
}

}  // namespace pwa
