// pwa_internal.h -- model state and kernel launchers shared by the library's
// translation units.  Not part of the public ABI (include/pwa.h is).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pwa.h"

namespace pwa {

// Events per tile of the tiled table layout (see k_table.hip).
constexpr int kTileEvents = 16;

// Stored entries of the tiled tables.  T_i is Hermitian, so its diagonal is
// real: the W diagonal entries are stored in pairs, (T_2d,2d, T_2d+1,2d+1) as
// the real and imaginary part of one complex entry d < D = ceil(W / 2) (the
// imaginary part is zero for the last entry of an odd W), followed by the
// W(W - 1)/2 entries a < b in row-major order.  A descriptor per stored entry
// says which: kDiagPair | a | a2 << 16 for a diagonal pair (a2 = kNoWave when
// there is none), a | b << 16 for an off-diagonal entry.  With this layout an
// entry's contribution to I_i is Re(c_e T_ie) for both kinds: c_e = 2 V_a V*_b
// off the diagonal and c_e = |V_a|^2 - i |V_a2|^2 for a diagonal pair.
constexpr uint32_t kDiagPair = 1u << 31;
constexpr uint32_t kNoWave = 0x7fffu;
__host__ __device__ inline int tiled_diag_entries(int W) { return (W + 1) / 2; }
__host__ __device__ inline int tiled_entries(int W) { return (W + 1) / 2 + W * (W - 1) / 2; }
// stored index of the off-diagonal entry (a, b), a < b
__host__ __device__ inline int tiled_offdiag_index(int W, int a, int b)
{
    return (W + 1) / 2 + a * (W - 1) - a * (a - 1) / 2 + (b - a - 1);
}

// Events per tile of the FP32 amplitude layout (padding unit).
constexpr int kAmpTile = 64;
constexpr size_t kLdsBytes = 160 * 1024;   // LDS per CU (gfx950)
// Events per tile of the 16-bit matrix-core layout (two MFMA rows each).
constexpr int kMfmaTile = 16;
// 16-bit elements of one tile of the matrix forms' adjoint operand copy, for
// KD = 2W rounded up to 16: full blocks of 32 rows x 32 slots, and when KD is
// an odd multiple of 16 a last block of 16 rows in the 16x16x32 operand order
// (512 elements)
__host__ __device__ constexpr int mfma_at_tile_elems(int kd)
{
    return ((kd / 16) & 1) ? (kd / 32) * 1024 + 512 : (kd / 32) * 1024;
}

// Lane-split layout of the FP32 amplitude form (k_amp.hip): an event is held
// by q = 2^lq neighbouring lanes with wl (even) waves each, so rows are q wl
// waves long.  The default shape minimises the padded row length, counted 25 %
// longer when wl > 10 (the registers of such lanes leave one wavefront per
// SIMD); among equal costs, the largest wl up to 10, else the smallest.
constexpr int kAmpMaxLaneWaves = 16;
struct AmpShape {
    int lq, wl;
};
__host__ __device__ inline AmpShape amp_shape(int W)
{
    AmpShape best{0, 0};
    int best_cost = 1 << 30;
    for (int lq = 0; lq <= 4; ++lq) {
        const int q = 1 << lq;
        int wl = (W + q - 1) / q;
        wl += wl & 1;
        if (wl < 2) wl = 2;
        if (wl > kAmpMaxLaneWaves) continue;
        const int cost = q * wl * (wl > 10 ? 5 : 4);
        bool take = cost < best_cost;
        if (cost == best_cost) {
            const bool cur_small = best.wl <= 10, new_small = wl <= 10;
            take = (new_small && (!cur_small || wl > best.wl)) || (!new_small && !cur_small && wl < best.wl);
        }
        if (take) {
            best_cost = cost;
            best = AmpShape{lq, wl};
        }
    }
    return best;
}

enum Form : uint32_t {
    kTable32 = PWA_FORM_TABLE,
    kAmp32 = PWA_FORM_AMPLITUDE,
    kTable64Plain = PWA_PRECISION_FP64_PLAIN,
    kTable64Fused = PWA_PRECISION_FP64_FUSED,
    kAmpBF16 = PWA_FORM_AMPLITUDE_BF16,
    kAmpFP16 = PWA_FORM_AMPLITUDE_FP16,
};

// Parameter vector passed by value in the kernel arguments: no host-to-device
// copy is needed per evaluation.  The asynchronous entry points set `dev`
// instead: V is then read from device memory when the kernel runs (so that a
// captured graph picks up new values on every replay).
struct VParams {
    double v[2 * PWA_MAX_WAVES_AMPLITUDE];
    const double* dev = nullptr;
};

// Where a kernel reads V from.
__device__ inline const double* vsrc(const VParams& vp) { return vp.dev ? vp.dev : vp.v; }

// Optional timing of a launch: when non-null, the runtime stamps `start` and
// `stop` with the begin and end times of the dispatch itself
// (hipExtLaunchKernel), so the elapsed time excludes launch latency.
struct LaunchEvents {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};

struct Model {
    int device = 0;
    Form form = kTable32;
    int64_t n = 0;           // data events
    int32_t W = 0;           // waves
    int32_t P = 0;           // packed entries W(W+1)/2 (the canonical table)
    int32_t ps = 0;          // stored entries per event of the main kernel's table layout
    int32_t wpad = 0;        // amplitude row length q wl (FP32 amplitude form)
    int32_t amp_lq = 0;      // FP32 amplitude form: log2 of the lanes per event
    int32_t amp_wl = 2;      // FP32 amplitude form: waves per lane
    int64_t n_tiles = 0;     // tiles of the main kernel's layout
    int32_t grid = 0;        // blocks of the main kernel
    int32_t cus = 0;         // compute units of the device
    int32_t rows = 0;        // partial records written per evaluation
    int32_t rec_len = 0;     // doubles per partial record
    int32_t kslots = 0;      // fused table kernel: slots of 64 entries per lane
    int32_t subtile = 0;     // fused table kernel: events per sub-tile
    int32_t amp_waves = 1;   // amplitude kernel: wavefronts per block

    void* d_data = nullptr;         // table (tiled or SoA) or padded amplitudes
    int64_t data_bytes = 0;
    uint32_t* d_pairs = nullptr;    // (a | a' << 16) per packed entry
    uint32_t* d_slots = nullptr;    // tiled tables: descriptor per stored entry
    double* d_M = nullptr;          // W x W complex128
    double* d_partials = nullptr;   // rows x rec_len
    double* d_colsum = nullptr;     // rec_len (x K for batched)
    double* d_w = nullptr;          // plain path: per-event weights 1/I_i
    double* h_out = nullptr;        // pinned host [nll, nbad, grad 2W] per evaluation
    unsigned long long* h_done = nullptr;   // pinned host completion words (one per assembly block)
    unsigned long long seq = 0;     // last published completion value
    int32_t out_cap = 1;            // evaluations h_out can hold

    int timing = 0;        // time every timing-th evaluation (0: none)
    int64_t timing_count = 0;
    // kernel timing: a ring of event pairs, read back only when a slot is
    // reused or the totals are asked for (no host wait per evaluation)
    static constexpr int kTimingRing = 64;
    hipEvent_t ev_start[kTimingRing] = {};
    hipEvent_t ev_stop[kTimingRing] = {};
    int ev_next = 0;       // slot of the next timed launch
    int ev_pending = 0;    // timed launches not read back yet (the slots before ev_next)
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
    double build_table_ms = 0.0;   // device time of the table (or amplitude) preparation
    double build_mc_ms = 0.0;      // device time of the MC integral M

    // 16-bit amplitude forms (matrix-core kernel, any number of vectors)
    void* d_at = nullptr;           // second copy of the event tiles (adjoint operand order)
    int32_t kd = 0;                 // row length 2W padded to a multiple of 16
    int32_t rb = 0;                 // adjoint row blocks of 32 (ceil(kd / 32))
    bool fwd_merge = false;         // bf16 with 2W mod 16 in 1..8: the second V part's last
                                    // forward K-step rides in the first part's padding slots
    int32_t vec_cap = 0;            // vectors the per-call buffers below can hold
    double* d_vb = nullptr;         // vec_cap x vprep_len(W) per-vector values (device)
    double* h_vstage = nullptr;     // vec_cap x 2W parameter vectors (mapped host memory)
    void* d_vm = nullptr;           // split vector matrix
    double* d_hrec = nullptr;       // FUMILI matrix: per-block records
    double* h_hout = nullptr;       // FUMILI matrix: 2W x 2W result (pinned host)
    unsigned long long* h_hdone = nullptr;   // its completion words (pinned host)
    double* d_brec = nullptr;       // per-(chunk, column) records: FP64 sums, then FP32 G
    size_t brec_rows = 0;           // (chunk, column block) pairs d_brec can hold
    int32_t done_cap = 0;           // completion words h_done can hold
};

// Many evaluations (jobs), possibly of different FP32 amplitude models, in one
// launch of the amplitude kernel and one of the assembly.  All tables live in
// device memory; the parameter buffer starts with the completion value (one
// 8-byte word) followed by each job's V.
struct MultiJob {
    const void* amp;            // the model's padded complex64 amplitudes
    int64_t n_events;
    int32_t W, wpad;
    int32_t lq, wl;             // lane-split shape of the amplitudes
    int32_t v_off;              // offset of V in the parameter buffer (doubles)
    int32_t rec0, nrec;         // the job's records: units rec0 .. rec0 + nrec - 1
    int32_t out_off;            // offset of [nll, n_bad, grad] in the output (doubles)
    int32_t done_off;           // first of the job's 1 + W completion words
    int32_t pad;
    const double2* M;
};
struct MultiUnit {
    int32_t job, pad;
    int64_t k0, k1;             // steps (64 / q events each) of the job's amplitudes
};
struct AsmBlock {
    int32_t job, role;          // role 0: NLL; 1 + b: gradient component b
};
// Units are grouped by waves per lane (one kernel instance each).
constexpr int kMultiClasses = kAmpMaxLaneWaves / 2;
struct MultiClass {
    int unit_off, n_units, wl;
};
struct MultiLaunch {
    const MultiJob* jobs;
    const MultiUnit* units;
    const AsmBlock* asm_blocks;
    const double* params;
    double* recs;
    double* out;                // pinned host
    unsigned long long* done;   // pinned host
    int rec_stride, n_units, n_asm;
    int n_classes;
    MultiClass cls[kMultiClasses];
};

// Per-vector values the matrix-core assembly needs besides the records,
// vprep_len(W) doubles per vector: [s_k, mu_k, m (Re m_b, Im m_b for b < W),
// the remainders the 16-bit split leaves out of each entry of the scaled
// column (2W)], with m_b = sum_a V_a M_ab and mu_k = Re sum_b conj(V_b) m_b.
__host__ __device__ inline int vprep_len(int W) { return 4 * W + 2; }

// One call of the matrix-core path: K vectors, device buffers and outputs.
struct MfmaBatch {
    const double* v;            // K x 2W (device, or mapped host memory)
    double* vprep;              // K x vprep_len(W): scale, mu, V M, split remainders (device)
    void* vm;                   // split vector matrix (device)
    double* rec_d;              // chunks x n_cb x 32 x 2: sum ln I, n_bad (device)
    float* rec_g;               // chunks x n_cb x 32 x kd: G columns, Re/Im g_b (device)
    double* out;                // K x (2 + 2W) (pinned host)
    unsigned long long* done;   // K completion words (pinned host)
    unsigned long long seq;
    int K;
    int n_cb;                   // column blocks of 32 vectors
    int chunks;                 // event chunks
};

// ---- launchers (each returns the hipError_t of its launch) ----------------
// build step
hipError_t launch_pack_tiled(const void* src, bool src_is_table, bool src_c128, int64_t n,
                             int W, int ps, const uint32_t* slots, bool store_c128,
                             int64_t n_tiles, void* dst, hipStream_t s, const LaunchEvents& ev);
// counts the diagonal entries of a canonical packed source table whose
// imaginary part is not zero (a Hermitian table has none) into *count
hipError_t launch_check_table_diag(const void* src, bool c128, int64_t n, int W,
                                   unsigned long long* count, hipStream_t s);
hipError_t launch_pack_soa(const void* src, bool src_is_table, bool src_c128, int64_t n, int W,
                           int P, const uint32_t* pairs, double* dst, hipStream_t s);
hipError_t launch_pack_amp(const void* src, bool src_c128, int64_t n, int W, AmpShape sh,
                           int64_t n_pad, float* dst, hipStream_t s);
hipError_t launch_stream_read(const void* p, int64_t bytes, uint32_t* sink, int sink_len,
                              hipStream_t s, const LaunchEvents& ev);
hipError_t launch_table_read(const Model& m, uint32_t* sink, hipStream_t s,
                             const LaunchEvents& ev);
int table_read_threads(const Model& m);
hipError_t launch_unpack_tiled(const void* src, bool c128, int64_t n, int W,
                               const uint32_t* pairs, void* dst, hipStream_t s);
hipError_t launch_unpack_soa(const double* src, int64_t n, int P, double* dst, hipStream_t s);
// the MC integral on the FP64 matrix cores, for 2W <= 256: records of
// gram_mfma_record(W) doubles per block, summed by k_colsum, then expanded
int gram_mfma_tiles(int W);   // 0 when W is too large
int gram_mfma_record(int W);
int gram_mfma_rows(int64_t n_acc, int W);
hipError_t launch_gram_mfma(const void* mc, bool c128, int64_t n_acc, int W, double* records,
                            int rows, hipStream_t s, const LaunchEvents& ev);
hipError_t launch_expand_gram(const double* colsum, int W, int64_t n_gen, double* M,
                              hipStream_t s);
int plain_rows(int64_t n);

// evaluation
struct TailArgs;
hipError_t launch_table_fused(const Model& m, const VParams& vp, bool grad, hipStream_t s,
                   const LaunchEvents& ev);
hipError_t launch_plain(const Model& m, const VParams& vp, bool grad, hipStream_t s,
                   const LaunchEvents& ev);
hipError_t launch_amp_fused(const Model& m, const VParams& vp, bool grad, hipStream_t s,
                   const LaunchEvents& ev);
hipError_t launch_colsum(const double* partials, int rows, int cols, int stride, double* out,
                         hipStream_t s);
hipError_t launch_pack_mfma(const void* src, bool c128, int64_t n, int W, bool bf,
                            const Model& m, hipStream_t s);
hipError_t launch_unpack_mfma(const Model& m, float* dst, hipStream_t s);
hipError_t launch_unpack_amp(const void* src, int64_t n, int W, AmpShape sh, float* dst,
                             hipStream_t s);
hipError_t launch_mfma_batch(const Model& m, const MfmaBatch& b, hipStream_t s,
                             const LaunchEvents& ev);
int mfma_chunks(const Model& m, int n_cb);
size_t mfma_vm_bytes(const Model& m, int n_cb);
// allocation-free matrix-core evaluation (pwa_nll_batched_noalloc): a static
// device array of kNoAllocScratchBytes per device and the layout of one call in it
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
constexpr int kNoAllocMaxDevices = 64;
constexpr int kNoAllocMaxVectors = 1024;
struct NoAllocLayout {
    int n_cb, chunks;
    size_t vprep_off, vm_off, rec_d_off, rec_g_off;    // byte offsets in the scratch array
};
hipError_t noalloc_scratch(int device, void** out);
bool noalloc_layout(const Model& m, int K, NoAllocLayout* L);
hipError_t launch_assemble(const VParams& vp, const TailArgs& ta, hipStream_t s);
hipError_t launch_amp_multi_class(const MultiLaunch& ml, int c, hipStream_t s);
hipError_t launch_assemble_multi(const MultiLaunch& ml, hipStream_t s);
int amp_multi_class(int wl);
hipError_t launch_hessian(const Model& m, const VParams& vp, double* recs, double* out,
                          unsigned long long* done, unsigned long long seq, hipStream_t s);
int hess_rows(const Model& m);
int hess_rec_doubles(int W);
int hess_assemble_blocks(int W);
int assemble_blocks(int W, bool grad);

// occupancy-derived grid sizes
int table_fused_grid(const Model& m);
int amp_fused_grid(Model& m);
int select_kslots(int P, bool c128);
int default_subtile(int kslots, bool c128);
bool fused_shape_ok(const Model& m);

}  // namespace pwa
