// pwa_api.cpp -- the C ABI declared in include/pwa.h: argument checking,
// device memory ownership, the build step and the evaluation sequence.
//
// Evaluation sequence on the caller's stream (all device work is in kernels):
//   main kernel (fused table / plain two-pass / amplitude) -> per-block partials
//   k_assemble: block 0 sums ln I and forms NLL = -sum ln I + mu, block 1 + b
//   sums the entries gradient component b needs and forms it; results go to
//   pinned host memory, each block then sets its completion word
//   the host polls a completion word in pinned memory; nothing is copied
//   with a separate transfer.
// V travels in the kernel arguments, so nothing is copied host-to-device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pwa.h"
#include "pwa_internal.h"
#include "tail.h"

using pwa::Model;

namespace {

constexpr uint32_t kFormBits = PWA_FORM_TABLE | PWA_FORM_AMPLITUDE | PWA_PRECISION_FP64_PLAIN |
                               PWA_PRECISION_FP64_FUSED | PWA_FORM_AMPLITUDE_BF16 |
                               PWA_FORM_AMPLITUDE_FP16;

thread_local std::string g_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int device_fail(hipError_t e, const char* what)
{
    (void)hipGetLastError();
    const int code = (e == hipErrorOutOfMemory) ? PWA_ERR_OOM : PWA_ERR_DEVICE;
    return fail(code, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                           \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return device_fail(e_, #expr);    \
    } while (0)

bool is_device_ptr(const void* p)
{
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged ||
           attr.type == hipMemoryTypeUnified;
}

// Switches to the model's device for the lifetime of the object.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Device copy of a caller buffer (or the buffer itself when it is on the device).
struct Staged {
    const void* ptr = nullptr;
    void* owned = nullptr;
    ~Staged()
    {
        if (owned) (void)hipFree(owned);
    }
};

int stage(const void* src, size_t bytes, hipStream_t s, Staged& out)
{
    if (is_device_ptr(src)) {
        out.ptr = src;
        return PWA_OK;
    }
    HIP_TRY(hipMalloc(&out.owned, bytes));
    HIP_TRY(hipMemcpyAsync(out.owned, src, bytes, hipMemcpyHostToDevice, s));
    out.ptr = out.owned;
    return PWA_OK;
}

void release(Model* m)
{
    if (!m) return;
    DeviceGuard g(m->device);
    if (m->d_data) (void)hipFree(m->d_data);
    if (m->d_pairs) (void)hipFree(m->d_pairs);
    if (m->d_slots) (void)hipFree(m->d_slots);
    if (m->d_M) (void)hipFree(m->d_M);
    if (m->d_partials) (void)hipFree(m->d_partials);
    if (m->d_colsum) (void)hipFree(m->d_colsum);
    if (m->d_w) (void)hipFree(m->d_w);
    if (m->d_at) (void)hipFree(m->d_at);
    if (m->d_vb) (void)hipFree(m->d_vb);
    if (m->d_vm) (void)hipFree(m->d_vm);
    if (m->d_brec) (void)hipFree(m->d_brec);
    if (m->h_vstage) (void)hipHostFree(m->h_vstage);
    if (m->d_hrec) (void)hipFree(m->d_hrec);
    if (m->h_hout) (void)hipHostFree(m->h_hout);
    if (m->h_hdone) (void)hipHostFree(m->h_hdone);

    if (m->h_out) (void)hipHostFree(m->h_out);
    if (m->h_done) (void)hipHostFree(m->h_done);
    for (int k = 0; k < Model::kTimingRing; ++k) {
        if (m->ev_start[k]) (void)hipEventDestroy(m->ev_start[k]);
        if (m->ev_stop[k]) (void)hipEventDestroy(m->ev_stop[k]);
    }
    delete m;
}

// Pinned, device-visible, coherent host memory: the final kernel writes the
// results there directly, so no device-to-host copy is queued.
int alloc_out(Model* m, int cap)
{
    const size_t bytes = sizeof(double) * (size_t)(2 + 2 * m->W) * cap;
    if (m->h_out) (void)hipHostFree(m->h_out);
    m->h_out = nullptr;
    HIP_TRY(hipHostMalloc(&m->h_out, bytes, hipHostMallocCoherent | hipHostMallocMapped));
    m->out_cap = cap;
    return PWA_OK;
}

// Peak device memory of a build (bytes, an upper estimate): the staged input
// when it is on the host, the stored table or amplitudes, the MC input staged
// with the MC integral's block records, and the per-evaluation buffers.
double build_device_bytes(int64_t n, int32_t W, int64_t n_acc, uint32_t flags, bool data_on_host,
                          bool mc_on_host)
{
    const uint32_t form = flags & kFormBits;
    const double P = 0.5 * W * (W + 1.0);
    const double dn = (double)n;
    const double in_elem = (flags & PWA_DATA_COMPLEX128) ? 16.0 : 8.0;
    double b = data_on_host ? dn * ((flags & PWA_INPUT_IS_TABLE) ? P : W) * in_elem : 0.0;
    const double ntile = std::ceil(dn / 16.0) * 16.0;
    switch (form) {
    case PWA_FORM_TABLE: b += ntile * pwa::tiled_entries(W) * 8.0; break;
    case PWA_PRECISION_FP64_FUSED: b += ntile * pwa::tiled_entries(W) * 16.0; break;
    case PWA_PRECISION_FP64_PLAIN: b += dn * P * 16.0 + dn * 8.0; break;
    case PWA_FORM_AMPLITUDE_BF16:
    case PWA_FORM_AMPLITUDE_FP16: {
        const int kd = (2 * W + 15) / 16 * 16;
        b += ntile * 2.0 * kd * 2.0 + ntile / 16.0 * pwa::mfma_at_tile_elems(kd) * 2.0;
        break;
    }
    default: {   // FP32 amplitudes in the default lane-split shape
        const pwa::AmpShape sh = pwa::amp_shape(W);
        b += std::ceil(dn / pwa::kAmpTile) * pwa::kAmpTile * (double)(sh.wl << sh.lq) * 8.0;
        break;
    }
    }
    const double mc_elem = (flags & PWA_MC_COMPLEX128) ? 16.0 : 8.0;
    if (n_acc > 0) b += (mc_on_host ? (double)n_acc * W * mc_elem : 0.0) + (double)n_acc * 64.0;
    return b + 64.0 * 1024 * 1024;   // records, M and other small buffers
}

int build_model(const void* data, int64_t n, int32_t W, const void* mc, int64_t n_acc,
                int64_t n_gen, uint32_t flags, hipStream_t s, Model* m)
{
    {   // pre-flight: refuse a model that cannot fit before anything is allocated or copied
        size_t free_b = 0, total_b = 0;
        HIP_TRY(hipMemGetInfo(&free_b, &total_b));
        const double need = build_device_bytes(n, W, n_acc, flags, !is_device_ptr(data),
                                               n_acc > 0 && !is_device_ptr(mc));
        if (need > (double)free_b)
            return fail(PWA_ERR_OOM,
                        "the model needs about %.3g GB of device memory during its build, "
                        "%.3g GB are free (N = %lld, W = %d)",
                        need / 1e9, (double)free_b / 1e9, (long long)n, W);
    }
    const uint32_t form = flags & kFormBits;
    const bool in_table = flags & PWA_INPUT_IS_TABLE;
    const bool data_c128 = flags & PWA_DATA_COMPLEX128;
    const bool mc_c128 = flags & PWA_MC_COMPLEX128;

    HIP_TRY(hipGetDevice(&m->device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, m->device));
    m->cus = prop.multiProcessorCount;
    m->form = (pwa::Form)form;
    m->n = n;
    m->W = W;
    m->P = W * (W + 1) / 2;
    const int P = m->P;

    // (a, a') of every packed entry, row-major upper triangle
    std::vector<uint32_t> pairs;
    pairs.reserve(P);
    for (int a = 0; a < W; ++a)
        for (int b = a; b < W; ++b) pairs.push_back((uint32_t)a | ((uint32_t)b << 16));
    HIP_TRY(hipMalloc(&m->d_pairs, sizeof(uint32_t) * P));
    HIP_TRY(hipMemcpyAsync(m->d_pairs, pairs.data(), sizeof(uint32_t) * P, hipMemcpyHostToDevice, s));

    // build-step timing: events around the table preparation and the MC
    // integral kernels (the inputs are already on the device by then)
    hipEvent_t bt[4] = {nullptr, nullptr, nullptr, nullptr};
    struct EventsGuard {
        hipEvent_t* e;
        ~EventsGuard()
        {
            for (int k = 0; k < 4; ++k)
                if (e[k]) (void)hipEventDestroy(e[k]);
        }
    } bt_guard{bt};
    for (int k = 0; k < 4; ++k) HIP_TRY(hipEventCreate(&bt[k]));

    // ---- data: table or amplitudes on the device ----
    const size_t in_elem = data_c128 ? 16 : 8;
    const size_t in_bytes = (size_t)n * (in_table ? P : W) * in_elem;
    Staged sd;
    int rc = stage(data, in_bytes, s, sd);
    if (rc != PWA_OK) return rc;
    m->ps = P;
    if (in_table) {
        // a Hermitian table has a real diagonal
        unsigned long long* d_count = nullptr;
        HIP_TRY(hipMalloc(&d_count, sizeof(unsigned long long)));
        unsigned long long bad = 0;
        hipError_t e = hipMemsetAsync(d_count, 0, sizeof bad, s);
        if (e == hipSuccess) e = pwa::launch_check_table_diag(sd.ptr, data_c128, n, W, d_count, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&bad, d_count, sizeof bad, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(d_count);
        if (e != hipSuccess) return device_fail(e, "table diagonal check");
        if (bad)
            return fail(PWA_ERR_INVALID,
                        "the input table is not Hermitian: %llu diagonal entries have a non-zero "
                        "imaginary part", bad);
    }

    if (form == PWA_FORM_TABLE || form == PWA_PRECISION_FP64_FUSED) {
        const bool c128 = form == PWA_PRECISION_FP64_FUSED;
        // stored entries: diagonal pairs, then the off-diagonal upper triangle
        m->ps = pwa::tiled_entries(W);
        std::vector<uint32_t> desc;
        desc.reserve(m->ps);
        for (int a = 0; a < W; a += 2)
            desc.push_back(pwa::kDiagPair | (uint32_t)a |
                           ((uint32_t)(a + 1 < W ? a + 1 : (int)pwa::kNoWave) << 16));
        for (int a = 0; a < W; ++a)
            for (int b = a + 1; b < W; ++b) desc.push_back((uint32_t)a | ((uint32_t)b << 16));
        HIP_TRY(hipMalloc(&m->d_slots, sizeof(uint32_t) * m->ps));
        HIP_TRY(hipMemcpyAsync(m->d_slots, desc.data(), sizeof(uint32_t) * m->ps,
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));   // desc leaves scope
        m->n_tiles = (n + pwa::kTileEvents - 1) / pwa::kTileEvents;
        m->data_bytes = m->n_tiles * pwa::kTileEvents * (int64_t)m->ps * (c128 ? 16 : 8);
        HIP_TRY(hipMalloc(&m->d_data, m->data_bytes));
        HIP_TRY(pwa::launch_pack_tiled(sd.ptr, in_table, data_c128, n, W, m->ps, m->d_slots, c128,
                                       m->n_tiles, m->d_data, s, pwa::LaunchEvents{bt[0], bt[1]}));
        m->kslots = pwa::select_kslots(m->ps, c128);
        if (m->kslots < 0) return fail(PWA_ERR_INVALID, "n_waves %d too large for the table form", W);
        m->subtile = pwa::default_subtile(m->kslots, c128);
        if (const char* env = std::getenv("PWA_TABLE_SUBTILE")) {
            const int e = std::atoi(env);
            const int keep = m->subtile;
            m->subtile = e;
            if (!pwa::fused_shape_ok(*m)) m->subtile = keep;
        }
        m->grid = pwa::table_fused_grid(*m);
        m->rows = m->grid;
        m->rec_len = 2 + 2 * W;   // [sum ln I, n_bad, u_b = sum_a V_a U_ab]
    } else if (form == PWA_PRECISION_FP64_PLAIN) {
        m->data_bytes = (int64_t)n * P * 16;
        HIP_TRY(hipMalloc(&m->d_data, m->data_bytes));
        HIP_TRY(hipEventRecord(bt[0], s));
        HIP_TRY(pwa::launch_pack_soa(sd.ptr, in_table, data_c128, n, W, P, m->d_pairs,
                                     (double*)m->d_data, s));
        HIP_TRY(hipEventRecord(bt[1], s));
        HIP_TRY(hipMalloc(&m->d_w, sizeof(double) * n));
        m->rows = pwa::plain_rows(n);
        m->grid = m->rows;
        m->rec_len = 2 + 2 * P;
    } else if (form == PWA_FORM_AMPLITUDE_BF16 || form == PWA_FORM_AMPLITUDE_FP16) {
        m->kd = (2 * W + 15) / 16 * 16;
        m->rb = (m->kd + 31) / 32;
        m->fwd_merge = form == PWA_FORM_AMPLITUDE_BF16 && (2 * W) % 16 != 0 && (2 * W) % 16 <= 8;
        m->n_tiles = (n + pwa::kMfmaTile - 1) / pwa::kMfmaTile;
        m->data_bytes = m->n_tiles * 32 * (int64_t)m->kd * 2;   // 32 rows per tile
        const size_t at_bytes = (size_t)m->n_tiles * pwa::mfma_at_tile_elems(m->kd) * 2;
        HIP_TRY(hipMalloc(&m->d_data, m->data_bytes));
        HIP_TRY(hipMalloc(&m->d_at, at_bytes));
        // padding events, columns 2W .. kd and adjoint rows 2W .. 32 rb stay zero
        HIP_TRY(hipMemsetAsync(m->d_data, 0, m->data_bytes, s));
        HIP_TRY(hipMemsetAsync(m->d_at, 0, at_bytes, s));
        HIP_TRY(hipEventRecord(bt[0], s));
        HIP_TRY(pwa::launch_pack_mfma(sd.ptr, data_c128, n, W, form == PWA_FORM_AMPLITUDE_BF16, *m,
                                      s));
        HIP_TRY(hipEventRecord(bt[1], s));
        m->rows = 0;
        m->rec_len = 2 + 2 * W;
    } else {   // amplitude form
        const pwa::AmpShape sh = pwa::amp_shape(W);
        m->amp_lq = sh.lq;
        m->amp_wl = sh.wl;
        m->wpad = sh.wl << sh.lq;
        m->n_tiles = (n + pwa::kAmpTile - 1) / pwa::kAmpTile;
        const int64_t n_pad = m->n_tiles * pwa::kAmpTile;
        m->data_bytes = n_pad * m->wpad * 8;
        HIP_TRY(hipMalloc(&m->d_data, m->data_bytes));
        HIP_TRY(hipEventRecord(bt[0], s));
        HIP_TRY(pwa::launch_pack_amp(sd.ptr, data_c128, n, W, sh, n_pad, (float*)m->d_data, s));
        HIP_TRY(hipEventRecord(bt[1], s));
        m->grid = pwa::amp_fused_grid(*m);
        m->rows = m->grid;
        m->rec_len = 2 + 2 * W;
    }

    // ---- MC matrix ----
    HIP_TRY(hipMalloc(&m->d_M, sizeof(double) * 2 * W * W));
    // the MC integral on the FP64 matrix cores (real Gram tiles, 2W <= 256)
    if (pwa::gram_mfma_tiles(W) <= 0)
        return fail(PWA_ERR_INVALID, "W = %d is too wide for the MC integral", W);
    const int grec = pwa::gram_mfma_record(W);
    HIP_TRY(hipMalloc(&m->d_colsum, sizeof(double) * (size_t)std::max(std::max(m->rec_len, 2 * P), grec)));
    if (n_acc > 0) {
        Staged sm;
        rc = stage(mc, (size_t)n_acc * W * (mc_c128 ? 16 : 8), s, sm);
        if (rc != PWA_OK) return rc;
        const int grows = pwa::gram_mfma_rows(n_acc, W);
        double* gpart = nullptr;
        HIP_TRY(hipMalloc(&gpart, sizeof(double) * grec * (size_t)grows));
        hipError_t e = hipStreamSynchronize(s);   // the MC input staged
        // dispatch-stamped start of the first kernel, plain event after the last
        if (e == hipSuccess)
            e = pwa::launch_gram_mfma(sm.ptr, mc_c128, n_acc, W, gpart, grows, s,
                                      pwa::LaunchEvents{bt[2], nullptr});
        if (e == hipSuccess) e = pwa::launch_colsum(gpart, grows, grec, grec, m->d_colsum, s);
        if (e == hipSuccess) e = pwa::launch_expand_gram(m->d_colsum, W, n_gen, m->d_M, s);
        if (e == hipSuccess) e = hipEventRecord(bt[3], s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, bt[2], bt[3]);
        m->build_mc_ms = ms;
        (void)hipFree(gpart);
        if (e != hipSuccess) return device_fail(e, "MC matrix build");
    } else {
        HIP_TRY(hipMemsetAsync(m->d_M, 0, sizeof(double) * 2 * W * W, s));
    }

    if (m->rows > 0)
        HIP_TRY(hipMalloc(&m->d_partials, sizeof(double) * (size_t)m->rows * m->rec_len));

    const int nblk = pwa::assemble_blocks(W, true);
    HIP_TRY(hipHostMalloc((void**)&m->h_done, sizeof(unsigned long long) * nblk,
                          hipHostMallocCoherent | hipHostMallocMapped));
    for (int k = 0; k < nblk; ++k) m->h_done[k] = 0;
    m->done_cap = nblk;
    rc = alloc_out(m, 1);
    if (rc != PWA_OK) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    float tms = 0.f;
    HIP_TRY(hipEventElapsedTime(&tms, bt[0], bt[1]));
    m->build_table_ms = tms;
    return PWA_OK;
}

// Add the kernel time of the `count` oldest unread timed launches.
int read_timing(Model* m, int count)
{
    const int R = Model::kTimingRing;
    for (int k = 0; k < count; ++k) {
        const int slot = ((m->ev_next - m->ev_pending) % R + R) % R;
        HIP_TRY(hipEventSynchronize(m->ev_stop[slot]));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, m->ev_start[slot], m->ev_stop[slot]));
        m->timed_ms += ms;
        m->timed_launches += 1;
        --m->ev_pending;
    }
    return PWA_OK;
}

// Event pair for the next timed launch (reading back the oldest when the ring
// is full: that launch finished long ago).
int timing_slot(Model* m, pwa::LaunchEvents* ev)
{
    const int R = Model::kTimingRing;
    if (m->ev_pending == R) {
        const int rc = read_timing(m, 1);
        if (rc != PWA_OK) return rc;
    }
    const int slot = m->ev_next;
    ev->start = m->ev_start[slot];
    ev->stop = m->ev_stop[slot];
    m->ev_next = (slot + 1) % R;
    ++m->ev_pending;
    return PWA_OK;
}

// Whether this evaluation is one of the timed ones.
bool take_timing(Model* m)
{
    if (m->timing <= 0) return false;
    return (m->timing_count++ % m->timing) == 0;
}

int check_v(const double* v, int W)
{
    for (int k = 0; k < 2 * W; ++k)
        if (!std::isfinite(v[k])) return fail(PWA_ERR_NONFINITE_INPUT, "v[%d] is not finite", k);
    return PWA_OK;
}

// Enqueue one evaluation writing slot `slot` of h_out; returns the completion
// value the last block will publish in h_done.  With v_dev set (asynchronous
// entry points), V is read from device memory, the results go to out_dev and
// nothing is published.
int enqueue_eval(Model* m, const double* v, bool grad, int slot, hipStream_t s, bool timed,
                 unsigned long long* seq_out, int* nblk_out, const double* v_dev = nullptr,
                 double* out_dev = nullptr)
{
    pwa::VParams vp;
    std::memset(&vp, 0, sizeof vp);
    if (v_dev) vp.dev = v_dev;
    else std::memcpy(vp.v, v, sizeof(double) * 2 * m->W);
    pwa::TailArgs ta;
    ta.rec = m->d_partials;
    ta.rows = m->rows;
    ta.rec_len = m->rec_len;
    ta.M = (const double2*)m->d_M;
    ta.out = v_dev ? out_dev : m->h_out + (size_t)slot * (2 + 2 * m->W);
    ta.done = v_dev ? nullptr : m->h_done;
    ta.seq = ++m->seq;
    ta.W = m->W;
    ta.grad = grad ? 1 : 0;
    ta.g_records = m->form == pwa::kTable64Plain ? 0 : 1;
    pwa::LaunchEvents ev;
    if (timed) {
        const int rc = timing_slot(m, &ev);
        if (rc != PWA_OK) return rc;
    }
    hipError_t e;
    if (m->form == pwa::kTable32 || m->form == pwa::kTable64Fused)
        e = pwa::launch_table_fused(*m, vp, grad, s, ev);
    else if (m->form == pwa::kTable64Plain)
        e = pwa::launch_plain(*m, vp, grad, s, ev);
    else
        e = pwa::launch_amp_fused(*m, vp, grad, s, ev);
    if (e != hipSuccess) return device_fail(e, "kernel launch");
    e = pwa::launch_assemble(vp, ta, s);
    if (e != hipSuccess) return device_fail(e, "assembly launch");
    *seq_out = ta.seq;
    *nblk_out = pwa::assemble_blocks(m->W, grad);
    return PWA_OK;
}

// Wait until the evaluation that publishes `seq` has written its results to
// host memory: every assembly block stores `seq` in its completion word after
// its outputs.  The host polls the words; every few thousand polls it asks the
// runtime whether the stream failed or finished without them.
int wait_for(Model* m, unsigned long long seq, int nblk, hipStream_t s)
{
    volatile unsigned long long* done = m->h_done;
    auto all_done = [&]() {
        for (int k = 0; k < nblk; ++k)
            if (done[k] != seq) return false;
        return true;
    };
    for (unsigned long it = 1;; ++it) {
        if (all_done()) break;
        if ((it & 4095) == 0) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                if (all_done()) break;
                return fail(PWA_ERR_DEVICE, "evaluation finished without publishing its result");
            }
            if (e != hipErrorNotReady) return device_fail(e, "evaluation");
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return PWA_OK;
}

bool is_mfma(const Model* m) { return m->form == pwa::kAmpBF16 || m->form == pwa::kAmpFP16; }

// ---- many evaluations of FP32 amplitude models in one launch ---------------
// A plan holds the work list of one set of (model, vector count) pairs, its
// device tables, the pinned parameter staging and a graph captured once:
// [copy parameters to the device, amplitude kernel over all work units,
// assembly of all evaluations].  Each call writes the new parameters and
// completion value into the staging buffer and replays the graph.  The last
// plan is kept for the next call with the same pairs; freeing one of its
// models discards it.
struct MultiPlan {
    std::vector<std::pair<const Model*, int>> key;
    int device = 0;
    int n_jobs = 0;
    std::vector<int32_t> job_w, out_off, v_off;
    void* d_tables = nullptr;
    double* d_params = nullptr;
    double* h_params = nullptr;
    size_t params_bytes = 0;
    double* d_recs = nullptr;
    double* h_out = nullptr;
    unsigned long long* h_done = nullptr;
    int n_done = 0;
    pwa::MultiLaunch ml{};
    hipStream_t cap = nullptr;
    hipStream_t side[pwa::kMultiClasses] = {};   // branches of the graph, one per class
    hipEvent_t fork = nullptr;
    hipEvent_t join[pwa::kMultiClasses] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned long long seq = 0;
};

// Plans in most-recently-used order; a call whose (model, K) list matches a
// cached plan replays it, so that alternating model sets (several pwa.Batch
// objects) never recapture.  At most kMaxPlans are kept.
constexpr size_t kMaxPlans = 8;
std::mutex g_plan_mu;
std::vector<MultiPlan*> g_plans;

void destroy_plan(MultiPlan* p)
{
    if (!p) return;
    DeviceGuard g(p->device);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    for (int c = 0; c < pwa::kMultiClasses; ++c) {
        if (p->side[c]) (void)hipStreamDestroy(p->side[c]);
        if (p->join[c]) (void)hipEventDestroy(p->join[c]);
    }
    if (p->fork) (void)hipEventDestroy(p->fork);
    if (p->d_tables) (void)hipFree(p->d_tables);
    if (p->d_params) (void)hipFree(p->d_params);
    if (p->d_recs) (void)hipFree(p->d_recs);
    if (p->h_params) (void)hipHostFree(p->h_params);
    if (p->h_out) (void)hipHostFree(p->h_out);
    if (p->h_done) (void)hipHostFree(p->h_done);
    delete p;
}

bool multi_eligible(pwa_model* const* models, int n_models, const int32_t* k_per_model)
{
    int jobs = 0;
    int dev = -1;
    for (int mi = 0; mi < n_models; ++mi) {
        const Model* m = reinterpret_cast<const Model*>(models[mi]);
        if (m->form != pwa::kAmp32) return false;
        if (dev >= 0 && m->device != dev) return false;
        dev = m->device;
        jobs += k_per_model[mi];
    }
    return jobs >= 2;
}

int build_plan(pwa_model* const* models, int n_models, const int32_t* k_per_model, MultiPlan** out)
{
    MultiPlan* p = new (std::nothrow) MultiPlan();
    if (!p) return fail(PWA_ERR_OOM, "host allocation failed");
    struct Guard {
        MultiPlan*& p;
        ~Guard() { destroy_plan(p); }
    } guard{p};
    std::vector<pwa::MultiJob> jobs;
    std::vector<pwa::MultiUnit> units;
    std::vector<pwa::AsmBlock> asmb;
    int wmax = 1;
    int64_t total_bytes = 0;
    std::vector<const Model*> job_model;
    int32_t out_off = 0, done_off = 0, v_off = 1;   // the completion value comes first
    for (int mi = 0; mi < n_models; ++mi) {
        const Model* m = reinterpret_cast<const Model*>(models[mi]);
        p->key.emplace_back(m, k_per_model[mi]);
        p->device = m->device;
        for (int k = 0; k < k_per_model[mi]; ++k) {
            pwa::MultiJob j{};
            j.amp = m->d_data;
            j.n_events = m->n;
            j.W = m->W;
            j.wpad = m->wpad;
            j.lq = m->amp_lq;
            j.wl = m->amp_wl;
            j.v_off = v_off;
            j.out_off = out_off;
            j.done_off = done_off;
            j.M = (const double2*)m->d_M;
            jobs.push_back(j);
            job_model.push_back(m);
            p->job_w.push_back(m->W);
            p->out_off.push_back(out_off);
            p->v_off.push_back(v_off);
            v_off += 2 * m->W;
            out_off += 2 + 2 * m->W;
            done_off += 1 + m->W;
            wmax = std::max<int>(wmax, m->W);
            total_bytes += m->data_bytes;
        }
    }
    p->n_jobs = (int)jobs.size();
    (void)total_bytes;
    // work units of about equal bytes within a class (one launch per class of
    // waves per lane), about 2048 per class and at least 256 KB and 16 steps
    // each; a unit is one block of the amplitude kernel, and the hardware hands
    // units to compute units as they free up
    std::vector<int64_t> class_bytes(pwa::kMultiClasses, 0);
    for (int ji = 0; ji < p->n_jobs; ++ji)
        class_bytes[pwa::amp_multi_class(job_model[ji]->amp_wl)] += job_model[ji]->data_bytes;
    std::vector<std::vector<pwa::MultiUnit>> by_class(pwa::kMultiClasses);
    for (int ji = 0; ji < p->n_jobs; ++ji) {
        const Model* m = job_model[ji];
        const int c = pwa::amp_multi_class(m->amp_wl);
        const int64_t unit_bytes = std::max<int64_t>(256 << 10, (class_bytes[c] + 2047) / 2048);
        const int64_t ns = m->n_tiles << m->amp_lq;
        const int64_t spu = std::max<int64_t>(16, unit_bytes / (512 * (int64_t)m->amp_wl));
        const int64_t nu = std::max<int64_t>(1, (ns + spu - 1) / spu);
        std::vector<pwa::MultiUnit>& cu = by_class[pwa::amp_multi_class(m->amp_wl)];
        jobs[ji].rec0 = (int32_t)cu.size();   // offset within its class for now
        jobs[ji].nrec = (int32_t)nu;
        for (int64_t u = 0; u < nu; ++u) {
            pwa::MultiUnit mu{};
            mu.job = ji;
            mu.k0 = u * ns / nu;
            mu.k1 = (u + 1) * ns / nu;
            cu.push_back(mu);
        }
        for (int r = 0; r <= jobs[ji].W; ++r) asmb.push_back(pwa::AsmBlock{ji, r});
    }
    pwa::MultiLaunch& ml = p->ml;
    ml.n_classes = pwa::kMultiClasses;
    std::vector<int> class_off(pwa::kMultiClasses, 0);
    for (int c = 0; c < pwa::kMultiClasses; ++c) {
        class_off[c] = (int)units.size();
        ml.cls[c] = pwa::MultiClass{(int)units.size(), (int)by_class[c].size(), 2 * c + 2};
        units.insert(units.end(), by_class[c].begin(), by_class[c].end());
    }
    for (int ji = 0; ji < p->n_jobs; ++ji)
        jobs[ji].rec0 += class_off[pwa::amp_multi_class(job_model[ji]->amp_wl)];
    DeviceGuard g(p->device);
    const size_t jb = sizeof(pwa::MultiJob) * jobs.size();
    const size_t ub = sizeof(pwa::MultiUnit) * units.size();
    const size_t ab = sizeof(pwa::AsmBlock) * asmb.size();
    HIP_TRY(hipMalloc(&p->d_tables, jb + ub + ab));
    char* t = (char*)p->d_tables;
    HIP_TRY(hipMemcpy(t, jobs.data(), jb, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(t + jb, units.data(), ub, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(t + jb + ub, asmb.data(), ab, hipMemcpyHostToDevice));
    p->params_bytes = sizeof(double) * (size_t)v_off;
    HIP_TRY(hipMalloc(&p->d_params, p->params_bytes));
    HIP_TRY(hipHostMalloc((void**)&p->h_params, p->params_bytes, hipHostMallocDefault));
    const int rec_stride = 2 + 2 * wmax;
    HIP_TRY(hipMalloc(&p->d_recs, sizeof(double) * rec_stride * units.size()));
    HIP_TRY(hipHostMalloc((void**)&p->h_out, sizeof(double) * out_off,
                          hipHostMallocCoherent | hipHostMallocMapped));
    HIP_TRY(hipHostMalloc((void**)&p->h_done, sizeof(unsigned long long) * done_off,
                          hipHostMallocCoherent | hipHostMallocMapped));
    for (int k = 0; k < done_off; ++k) p->h_done[k] = 0;
    p->n_done = done_off;
    ml.jobs = (const pwa::MultiJob*)t;
    ml.units = (const pwa::MultiUnit*)(t + jb);
    ml.asm_blocks = (const pwa::AsmBlock*)(t + jb + ub);
    ml.params = p->d_params;
    ml.recs = p->d_recs;
    ml.out = p->h_out;
    ml.done = p->h_done;
    ml.rec_stride = rec_stride;
    ml.n_units = (int)units.size();
    ml.n_asm = (int)asmb.size();
    // capture [parameter copy, one amplitude launch per class, assembly] once;
    // the class launches are independent branches of the graph
    HIP_TRY(hipStreamCreate(&p->cap));
    HIP_TRY(hipEventCreateWithFlags(&p->fork, hipEventDisableTiming));
    int first = -1;
    for (int c = 0; c < ml.n_classes; ++c) {
        if (ml.cls[c].n_units == 0) continue;
        if (first < 0) {
            first = c;
            continue;
        }
        HIP_TRY(hipStreamCreate(&p->side[c]));
        HIP_TRY(hipEventCreateWithFlags(&p->join[c], hipEventDisableTiming));
    }
    HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipMemcpyAsync(p->d_params, p->h_params, p->params_bytes, hipMemcpyHostToDevice,
                                  p->cap);
    if (e == hipSuccess) e = hipEventRecord(p->fork, p->cap);
    for (int c = 0; c < ml.n_classes && e == hipSuccess; ++c) {
        if (!p->side[c]) continue;
        e = hipStreamWaitEvent(p->side[c], p->fork, 0);
        if (e == hipSuccess) e = pwa::launch_amp_multi_class(ml, c, p->side[c]);
        if (e == hipSuccess) e = hipEventRecord(p->join[c], p->side[c]);
    }
    if (e == hipSuccess && first >= 0) e = pwa::launch_amp_multi_class(ml, first, p->cap);
    for (int c = 0; c < ml.n_classes && e == hipSuccess; ++c)
        if (p->join[c]) e = hipStreamWaitEvent(p->cap, p->join[c], 0);
    if (e == hipSuccess) e = pwa::launch_assemble_multi(ml, p->cap);
    const hipError_t e2 = hipStreamEndCapture(p->cap, &p->graph);
    if (e != hipSuccess) return device_fail(e, "multi-evaluation capture");
    if (e2 != hipSuccess) return device_fail(e2, "multi-evaluation capture");
    HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    *out = p;
    p = nullptr;   // the guard releases nothing
    return PWA_OK;
}

// Run every (model, vector) evaluation of the call through the cached plan.
int eval_multi(pwa_model* const* models, int n_models, const int32_t* k_per_model,
               const double* v, double* nll, double* grad, hipStream_t s)
{
    std::lock_guard<std::mutex> lock(g_plan_mu);
    auto matches = [&](const MultiPlan* q) {
        if ((int)q->key.size() != n_models) return false;
        for (int mi = 0; mi < n_models; ++mi)
            if (q->key[mi].first != reinterpret_cast<const Model*>(models[mi]) ||
                q->key[mi].second != k_per_model[mi])
                return false;
        return true;
    };
    size_t hit = g_plans.size();
    for (size_t i = 0; i < g_plans.size(); ++i)
        if (matches(g_plans[i])) {
            hit = i;
            break;
        }
    MultiPlan* p = nullptr;
    if (hit < g_plans.size()) {
        p = g_plans[hit];
        g_plans.erase(g_plans.begin() + (std::ptrdiff_t)hit);
    } else {
        const int rc = build_plan(models, n_models, k_per_model, &p);
        if (rc != PWA_OK) return rc;
        if (g_plans.size() >= kMaxPlans) {
            destroy_plan(g_plans.back());
            g_plans.pop_back();
        }
    }
    g_plans.insert(g_plans.begin(), p);
    DeviceGuard g(p->device);
    const unsigned long long seq = ++p->seq;
    std::memcpy(p->h_params, &seq, sizeof seq);
    size_t vpos = 0;
    for (int j = 0; j < p->n_jobs; ++j) {
        std::memcpy(p->h_params + p->v_off[j], v + vpos, sizeof(double) * 2 * p->job_w[j]);
        vpos += 2 * p->job_w[j];
    }
    HIP_TRY(hipGraphLaunch(p->exec, s));
    volatile unsigned long long* done = p->h_done;
    for (unsigned long it = 1;; ++it) {
        bool all = true;
        for (int k = 0; k < p->n_done && all; ++k) all = done[k] == seq;
        if (all) break;
        if ((it & 4095) == 0) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                bool again = true;
                for (int k = 0; k < p->n_done && again; ++k) again = done[k] == seq;
                if (again) break;
                return fail(PWA_ERR_DEVICE, "evaluation finished without publishing its result");
            }
            if (e != hipErrorNotReady) return device_fail(e, "multi-model evaluation");
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    int status = PWA_OK;
    size_t gpos = 0;
    for (int j = 0; j < p->n_jobs; ++j) {
        const double* o = p->h_out + p->out_off[j];
        nll[j] = o[0];
        if (grad) std::memcpy(grad + gpos, o + 2, sizeof(double) * 2 * p->job_w[j]);
        gpos += 2 * p->job_w[j];
        if (o[1] > 0.0) status = PWA_WARN_DEGENERATE;
    }
    return status;
}

// Discard the cached plans that refer to model m.
void forget_model(const Model* m)
{
    std::lock_guard<std::mutex> lock(g_plan_mu);
    for (size_t i = 0; i < g_plans.size();) {
        bool uses = false;
        for (const auto& kv : g_plans[i]->key) uses = uses || kv.first == m;
        if (uses) {
            destroy_plan(g_plans[i]);
            g_plans.erase(g_plans.begin() + (std::ptrdiff_t)i);
        } else {
            ++i;
        }
    }
}

// Per-call buffers of the matrix-core path, grown to hold K vectors.
int mfma_reserve(Model* m, int K, int n_cb, int chunks)
{
    const int W = m->W;
    if (K > m->vec_cap) {
        const int cap = (K + 15) / 16 * 16;
        if (m->d_vb) (void)hipFree(m->d_vb);
        if (m->h_vstage) (void)hipHostFree(m->h_vstage);
        if (m->d_vm) (void)hipFree(m->d_vm);
        if (m->d_brec) (void)hipFree(m->d_brec);
        m->d_vb = nullptr;
        m->h_vstage = nullptr;
        m->d_vm = nullptr;
        m->d_brec = nullptr;
        m->vec_cap = 0;
        const int cb_cap = (cap + 31) / 32;
        HIP_TRY(hipMalloc(&m->d_vb, sizeof(double) * pwa::vprep_len(W) * (size_t)cap));
        // the vectors, read by the kernels straight from mapped host memory
        HIP_TRY(hipHostMalloc((void**)&m->h_vstage, sizeof(double) * 2 * W * (size_t)cap,
                              hipHostMallocCoherent | hipHostMallocMapped));
        HIP_TRY(hipMalloc(&m->d_vm, pwa::mfma_vm_bytes(*m, cb_cap)));
        // chunks x column blocks stays near 2048 (or below) for every K up to cap
        size_t rec_rows = 0;
        for (int cb = 1; cb <= cb_cap; ++cb) {
            const size_t r = (size_t)pwa::mfma_chunks(*m, cb) * cb;
            if (r > rec_rows) rec_rows = r;
        }
        HIP_TRY(hipMalloc(&m->d_brec, rec_rows * 32 * (2 * sizeof(double) + sizeof(float) * m->kd)));
        m->brec_rows = rec_rows;
        m->vec_cap = cap;
    }
    (void)n_cb;
    (void)chunks;
    if (K > m->out_cap) {
        const int rc = alloc_out(m, K);
        if (rc != PWA_OK) return rc;
    }
    if (K > m->done_cap) {
        if (m->h_done) (void)hipHostFree(m->h_done);
        m->h_done = nullptr;
        m->done_cap = 0;
        HIP_TRY(hipHostMalloc((void**)&m->h_done, sizeof(unsigned long long) * K,
                              hipHostMallocCoherent | hipHostMallocMapped));
        for (int k = 0; k < K; ++k) m->h_done[k] = 0;
        m->done_cap = K;
    }
    return PWA_OK;
}

// K evaluations on a 16-bit amplitude model in one pass; results in
// h_out[k * (2 + 2W)].
int eval_mfma(Model* m, const double* v, int K, hipStream_t s, bool timed)
{
    const int W = m->W;
    const int n_cb = (K + 31) / 32;
    const int chunks = pwa::mfma_chunks(*m, n_cb);
    int rc = mfma_reserve(m, K, n_cb, chunks);
    if (rc != PWA_OK) return rc;
    // the previous call has finished (its results were awaited), so no
    // kernel still reads the staging buffer
    std::memcpy(m->h_vstage, v, sizeof(double) * 2 * W * (size_t)K);
    pwa::MfmaBatch b;
    b.v = m->h_vstage;
    b.vprep = m->d_vb;
    b.vm = m->d_vm;
    b.rec_d = m->d_brec;
    b.rec_g = (float*)(m->d_brec + 2 * 32 * m->brec_rows);
    b.out = m->h_out;
    b.done = m->h_done;
    b.seq = ++m->seq;
    b.K = K;
    b.n_cb = n_cb;
    b.chunks = chunks;
    pwa::LaunchEvents ev;
    if (timed) {
        rc = timing_slot(m, &ev);
        if (rc != PWA_OK) return rc;
    }
    const hipError_t e = pwa::launch_mfma_batch(*m, b, s, ev);
    if (e != hipSuccess) return device_fail(e, "matrix-core evaluation launch");
    return wait_for(m, b.seq, K, s);
}

// Wait until all n words hold seq (see wait_for).
int poll_words(volatile unsigned long long* words, int n, unsigned long long seq, hipStream_t s)
{
    auto all_done = [&]() {
        for (int k = 0; k < n; ++k)
            if (words[k] != seq) return false;
        return true;
    };
    for (unsigned long it = 1;; ++it) {
        if (all_done()) break;
        if ((it & 4095) == 0) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                if (all_done()) break;
                return fail(PWA_ERR_DEVICE, "evaluation finished without publishing its result");
            }
            if (e != hipErrorNotReady) return device_fail(e, "evaluation");
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return PWA_OK;
}

int evaluate(const pwa_model* cm, const double* v, double* nll, double* grad, void* stream)
{
    if (!cm || !v || !nll) return fail(PWA_ERR_INVALID, "NULL model, v or nll");
    Model* m = reinterpret_cast<Model*>(const_cast<pwa_model*>(cm));
    int rc = check_v(v, m->W);
    if (rc != PWA_OK) return rc;
    DeviceGuard g(m->device);
    hipStream_t s = (hipStream_t)stream;
    const bool want_grad = grad != nullptr;
    if (is_mfma(m)) {
        rc = eval_mfma(m, v, 1, s, take_timing(m));
    } else {
        unsigned long long seq = 0;
        int nblk = 0;
        rc = enqueue_eval(m, v, want_grad, 0, s, take_timing(m), &seq, &nblk);
        if (rc != PWA_OK) return rc;
        rc = wait_for(m, seq, nblk, s);
    }
    if (rc != PWA_OK) return rc;
    *nll = m->h_out[0];
    if (want_grad) std::memcpy(grad, m->h_out + 2, sizeof(double) * 2 * m->W);
    return m->h_out[1] > 0.0 ? PWA_WARN_DEGENERATE : PWA_OK;
}

}  // namespace

// Re-store the FP32 amplitudes of m in shape sh (through a row-major copy).
int reshape_amp(Model* m, pwa::AmpShape sh, hipStream_t s)
{
    if (sh.lq == m->amp_lq && sh.wl == m->amp_wl) return PWA_OK;
    forget_model(m);   // a cached multi-model plan holds the old layout
    const int64_t n_pad = m->n_tiles * pwa::kAmpTile;
    const int64_t new_bytes = n_pad * ((int64_t)sh.wl << sh.lq) * 8;
    void* tmp = nullptr;
    void* nd = nullptr;
    HIP_TRY(hipMalloc(&tmp, std::max<size_t>(8, (size_t)m->n * m->W * 8)));
    hipError_t e = hipMalloc(&nd, new_bytes);
    if (e == hipSuccess)
        e = pwa::launch_unpack_amp(m->d_data, m->n, m->W, pwa::AmpShape{m->amp_lq, m->amp_wl},
                                   (float*)tmp, s);
    if (e == hipSuccess) e = pwa::launch_pack_amp(tmp, false, m->n, m->W, sh, n_pad, (float*)nd, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (e != hipSuccess) {
        if (nd) (void)hipFree(nd);
        return device_fail(e, "amplitude re-store");
    }
    (void)hipFree(m->d_data);
    m->d_data = nd;
    m->data_bytes = new_bytes;
    m->amp_lq = sh.lq;
    m->amp_wl = sh.wl;
    m->wpad = sh.wl << sh.lq;
    const int old_rows = m->rows;
    m->grid = pwa::amp_fused_grid(*m);
    m->rows = m->grid;
    if (m->rows > old_rows) {
        (void)hipFree(m->d_partials);
        m->d_partials = nullptr;
        HIP_TRY(hipMalloc(&m->d_partials, sizeof(double) * (size_t)m->rows * m->rec_len));
    }
    return PWA_OK;
}

bool valid_shape(int W, int lanes, int wl)
{
    const bool pow2 = lanes == 1 || lanes == 2 || lanes == 4 || lanes == 8 || lanes == 16;
    return pow2 && wl >= 2 && wl <= pwa::kAmpMaxLaneWaves && (wl % 2) == 0 && lanes * wl >= W;
}

int log2_lanes(int lanes)
{
    int lq = 0;
    while ((1 << lq) < lanes) ++lq;
    return lq;
}

// The asynchronous twins: enqueue only (kernels, nothing allocated, no host
// memory touched), so that the work can be captured in a graph.
int evaluate_async(const pwa_model* cm, const double* v_dev, double* out_dev, bool grad,
                   void* stream)
{
    if (!cm || !v_dev || !out_dev) return fail(PWA_ERR_INVALID, "NULL model, v_dev or out_dev");
    Model* m = reinterpret_cast<Model*>(const_cast<pwa_model*>(cm));
    if (is_mfma(m))
        return fail(PWA_ERR_INVALID, "the asynchronous entry points do not take the 16-bit forms");
    DeviceGuard g(m->device);
    unsigned long long seq = 0;
    int nblk = 0;
    return enqueue_eval(m, nullptr, grad, 0, (hipStream_t)stream, false, &seq, &nblk, v_dev,
                        out_dev);
}

extern "C" {

int pwa_build_table(const void* data, int64_t n_data, int32_t n_waves, const void* mc_amp,
                    int64_t n_mc_acc, int64_t n_mc_gen, uint32_t flags, void* hip_stream,
                    pwa_model** out)
{
    if (!out) return fail(PWA_ERR_INVALID, "out is NULL");
    *out = nullptr;
    const uint32_t known = kFormBits | PWA_INPUT_IS_TABLE | PWA_DATA_COMPLEX128 | PWA_MC_COMPLEX128;
    if (flags & ~known) return fail(PWA_ERR_INVALID, "unknown flag bits 0x%x", flags & ~known);
    const uint32_t form = flags & kFormBits;
    if (form == 0 || (form & (form - 1)) != 0)
        return fail(PWA_ERR_INVALID, "exactly one form flag is required (got 0x%x)", form);
    const bool amp_form = form == PWA_FORM_AMPLITUDE || form == PWA_FORM_AMPLITUDE_BF16 ||
                          form == PWA_FORM_AMPLITUDE_FP16;
    if (!data) return fail(PWA_ERR_INVALID, "data is NULL");
    if (n_data < 1) return fail(PWA_ERR_INVALID, "n_data must be >= 1 (got %lld)", (long long)n_data);
    const int wmax = form == PWA_FORM_AMPLITUDE ? PWA_MAX_WAVES_AMPLITUDE
                     : amp_form             ? PWA_MAX_WAVES_MATRIX
                                            : PWA_MAX_WAVES_TABLE;
    if (n_waves < 1 || n_waves > wmax)
        return fail(PWA_ERR_INVALID, "n_waves must be in [1, %d] for this form (got %d)", wmax, n_waves);
    if ((flags & PWA_INPUT_IS_TABLE) && amp_form)
        return fail(PWA_ERR_INVALID, "PWA_INPUT_IS_TABLE needs a table form");
    if (n_mc_acc < 0) return fail(PWA_ERR_INVALID, "n_mc_acc must be >= 0");
    if (n_mc_acc > 0 && !mc_amp) return fail(PWA_ERR_INVALID, "mc_amp is NULL but n_mc_acc > 0");
    if (n_mc_gen < 1) return fail(PWA_ERR_INVALID, "n_mc_gen must be >= 1");
    if (n_mc_acc > n_mc_gen) return fail(PWA_ERR_INVALID, "n_mc_acc exceeds n_mc_gen");
    if (n_data > ((int64_t)1 << 40)) return fail(PWA_ERR_INVALID, "n_data too large");

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return fail(PWA_ERR_NO_DEVICE, "no HIP device available");
    }
    Model* m = new (std::nothrow) Model();
    if (!m) return fail(PWA_ERR_OOM, "host allocation failed");
    const int rc = build_model(data, n_data, n_waves, mc_amp, n_mc_acc, n_mc_gen, flags,
                               (hipStream_t)hip_stream, m);
    if (rc != PWA_OK) {
        (void)hipStreamSynchronize((hipStream_t)hip_stream);
        release(m);
        return rc;
    }
    *out = reinterpret_cast<pwa_model*>(m);
    return PWA_OK;
}

int pwa_nll_grad_hess(const pwa_model* model, const double* v, double* nll, double* grad,
                      double* hess, void* hip_stream)
{
    if (!model || !v || !nll || !grad || !hess)
        return fail(PWA_ERR_INVALID, "NULL model, v, nll, grad or hess");
    Model* m = reinterpret_cast<Model*>(const_cast<pwa_model*>(model));
    if (m->form != pwa::kAmp32)
        return fail(PWA_ERR_INVALID, "the FUMILI matrix is computed for PWA_FORM_AMPLITUDE models");
    int rc = check_v(v, m->W);
    if (rc != PWA_OK) return rc;
    DeviceGuard g(m->device);
    hipStream_t s = (hipStream_t)hip_stream;
    const int W = m->W;
    const int nh = pwa::hess_assemble_blocks(W);
    if (!m->d_hrec) {
        HIP_TRY(hipMalloc(&m->d_hrec, sizeof(double) * (size_t)pwa::hess_rows(*m) *
                                          pwa::hess_rec_doubles(W)));
        HIP_TRY(hipHostMalloc((void**)&m->h_hout, sizeof(double) * 4 * W * W,
                              hipHostMallocCoherent | hipHostMallocMapped));
        HIP_TRY(hipHostMalloc((void**)&m->h_hdone, sizeof(unsigned long long) * nh,
                              hipHostMallocCoherent | hipHostMallocMapped));
        for (int k = 0; k < nh; ++k) m->h_hdone[k] = 0;
    }
    unsigned long long seq = 0;
    int nblk = 0;
    rc = enqueue_eval(m, v, true, 0, s, false, &seq, &nblk);
    if (rc != PWA_OK) return rc;
    pwa::VParams vp;
    std::memset(&vp, 0, sizeof vp);
    std::memcpy(vp.v, v, sizeof(double) * 2 * W);
    const unsigned long long hseq = ++m->seq;
    const hipError_t e = pwa::launch_hessian(*m, vp, m->d_hrec, m->h_hout, m->h_hdone, hseq, s);
    if (e != hipSuccess) return device_fail(e, "second-derivative launch");
    rc = poll_words(m->h_done, nblk, seq, s);
    if (rc != PWA_OK) return rc;
    rc = poll_words(m->h_hdone, nh, hseq, s);
    if (rc != PWA_OK) return rc;
    *nll = m->h_out[0];
    std::memcpy(grad, m->h_out + 2, sizeof(double) * 2 * W);
    std::memcpy(hess, m->h_hout, sizeof(double) * 4 * W * W);
    return m->h_out[1] > 0.0 ? PWA_WARN_DEGENERATE : PWA_OK;
}

int pwa_nll(const pwa_model* model, const double* v, double* nll, void* hip_stream)
{
    return evaluate(model, v, nll, nullptr, hip_stream);
}

int pwa_nll_grad(const pwa_model* model, const double* v, double* nll, double* grad,
                 void* hip_stream)
{
    if (!grad) return fail(PWA_ERR_INVALID, "grad is NULL");
    return evaluate(model, v, nll, grad, hip_stream);
}

int pwa_nll_async(const pwa_model* model, const double* v_dev, double* out_dev, void* hip_stream)
{
    return evaluate_async(model, v_dev, out_dev, false, hip_stream);
}

int pwa_nll_grad_async(const pwa_model* model, const double* v_dev, double* out_dev,
                       void* hip_stream)
{
    return evaluate_async(model, v_dev, out_dev, true, hip_stream);
}

int pwa_nll_batched_noalloc(const pwa_model* model, int32_t k, const double* v_dev,
                            double* out_dev, void* hip_stream)
{
    if (!model || !v_dev || !out_dev) return fail(PWA_ERR_INVALID, "NULL model, v_dev or out_dev");
    const Model* m = reinterpret_cast<const Model*>(model);
    if (!is_mfma(m))
        return fail(PWA_ERR_INVALID,
                    "pwa_nll_batched_noalloc takes the 16-bit amplitude forms only");
    if (k < 1 || k > pwa::kNoAllocMaxVectors)
        return fail(PWA_ERR_INVALID, "k must be in [1, %d] (got %d)", pwa::kNoAllocMaxVectors, k);
    pwa::NoAllocLayout L;
    if (!pwa::noalloc_layout(*m, k, &L))
        return fail(PWA_ERR_INVALID,
                    "%d vectors at W = %d need more than the %zu bytes of the static scratch", k,
                    m->W, pwa::kNoAllocScratchBytes);
    DeviceGuard g(m->device);
    void* base = nullptr;
    HIP_TRY(pwa::noalloc_scratch(m->device, &base));
    char* b8 = static_cast<char*>(base);
    pwa::MfmaBatch b;
    b.v = v_dev;
    b.vprep = reinterpret_cast<double*>(b8 + L.vprep_off);
    b.vm = b8 + L.vm_off;
    b.rec_d = reinterpret_cast<double*>(b8 + L.rec_d_off);
    b.rec_g = reinterpret_cast<float*>(b8 + L.rec_g_off);
    b.out = out_dev;
    b.done = nullptr;
    b.seq = 0;
    b.K = k;
    b.n_cb = L.n_cb;
    b.chunks = L.chunks;
    const hipError_t e = pwa::launch_mfma_batch(*m, b, (hipStream_t)hip_stream, pwa::LaunchEvents{});
    if (e != hipSuccess) return device_fail(e, "matrix-core evaluation launch");
    return PWA_OK;
}

int pwa_nll_batched(pwa_model* const* models, int32_t n_models, const int32_t* k_per_model,
                    const double* v, double* nll, double* grad, void* hip_stream)
{
    if (n_models < 0) return fail(PWA_ERR_INVALID, "n_models < 0");
    if (n_models == 0) return PWA_OK;
    if (!models || !k_per_model || !v || !nll)
        return fail(PWA_ERR_INVALID, "NULL models, k_per_model, v or nll");
    for (int mi = 0; mi < n_models; ++mi) {
        if (!models[mi]) return fail(PWA_ERR_INVALID, "models[%d] is NULL", mi);
        if (k_per_model[mi] < 0) return fail(PWA_ERR_INVALID, "k_per_model[%d] < 0", mi);
    }
    hipStream_t s = (hipStream_t)hip_stream;
    if (multi_eligible(models, n_models, k_per_model)) {
        const double* vq = v;
        for (int mi = 0; mi < n_models; ++mi) {
            const int W = reinterpret_cast<const Model*>(models[mi])->W;
            for (int k = 0; k < k_per_model[mi]; ++k, vq += 2 * W) {
                const int rc = check_v(vq, W);
                if (rc != PWA_OK) return rc;
            }
        }
        return eval_multi(models, n_models, k_per_model, v, nll, grad, s);
    }
    int status = PWA_OK;
    const double* vp = v;
    double* np = nll;
    double* gp = grad;
    for (int mi = 0; mi < n_models; ++mi) {
        Model* m = reinterpret_cast<Model*>(models[mi]);
        const int K = k_per_model[mi];
        const int W = m->W;
        for (int k = 0; k < K; ++k) {
            const int rc = check_v(vp + (size_t)k * 2 * W, W);
            if (rc != PWA_OK) return rc;
        }
        DeviceGuard g(m->device);
        if (is_mfma(m)) {
            if (K > 0) {
                const int rc = eval_mfma(m, vp, K, s, take_timing(m));
                if (rc != PWA_OK) return rc;
            }
        } else {
            if (K > m->out_cap) {
                const int rc = alloc_out(m, K);
                if (rc != PWA_OK) return rc;
            }
            unsigned long long seq = 0;
            int nblk = 0;
            for (int k = 0; k < K; ++k) {
                const int rc = enqueue_eval(m, vp + (size_t)k * 2 * W, gp != nullptr, k, s, false,
                                            &seq, &nblk);
                if (rc != PWA_OK) return rc;
            }
            if (K > 0) {
                const int rc = wait_for(m, seq, nblk, s);
                if (rc != PWA_OK) return rc;
            }
        }
        for (int k = 0; k < K; ++k) {
            const double* o = m->h_out + (size_t)k * (2 + 2 * W);
            np[k] = o[0];
            if (gp) std::memcpy(gp + (size_t)k * 2 * W, o + 2, sizeof(double) * 2 * W);
            if (o[1] > 0.0) status = PWA_WARN_DEGENERATE;
        }
        vp += (size_t)K * 2 * W;
        np += K;
        if (gp) gp += (size_t)K * 2 * W;
    }
    return status;
}

void pwa_free(pwa_model* model)
{
    if (!model) return;
    forget_model(reinterpret_cast<const Model*>(model));
    release(reinterpret_cast<Model*>(model));
}

const char* pwa_last_error(void)
{
    return g_error.c_str();
}

int pwa_model_info(const pwa_model* model, pwa_info* out)
{
    if (!model || !out) return fail(PWA_ERR_INVALID, "NULL model or out");
    const Model* m = reinterpret_cast<const Model*>(model);
    out->n_data = m->n;
    out->n_waves = m->W;
    out->n_packed = m->P;
    out->form = (uint32_t)m->form;
    switch (m->form) {
    case pwa::kTable32: out->stream_bytes = m->n * m->ps * 8; break;
    case pwa::kTable64Fused: out->stream_bytes = m->n * m->ps * 16; break;
    case pwa::kTable64Plain: out->stream_bytes = 2 * m->n * m->P * 16; break;
    case pwa::kAmpBF16:
    case pwa::kAmpFP16:
        out->stream_bytes = m->n_tiles * (int64_t)(32 * m->kd + pwa::mfma_at_tile_elems(m->kd)) * 2;   // both copies
        break;
    default: out->stream_bytes = m->n * m->W * 8; break;
    }
    out->grid_blocks = m->grid;
    out->compute_units = m->cus;
    return PWA_OK;
}

int pwa_copy_table(const pwa_model* model, void* out_host, void* hip_stream)
{
    if (!model || !out_host) return fail(PWA_ERR_INVALID, "NULL model or out_host");
    const Model* m = reinterpret_cast<const Model*>(model);
    DeviceGuard g(m->device);
    hipStream_t s = (hipStream_t)hip_stream;
    if (m->form == pwa::kAmp32) {   // the stored complex64 amplitudes, N x W
        const size_t bytes = (size_t)m->n * m->W * 8;
        void* tmp = nullptr;
        HIP_TRY(hipMalloc(&tmp, std::max<size_t>(bytes, 8)));
        hipError_t e = pwa::launch_unpack_amp(m->d_data, m->n, m->W,
                                              pwa::AmpShape{m->amp_lq, m->amp_wl}, (float*)tmp, s);
        if (e == hipSuccess) e = hipMemcpyAsync(out_host, tmp, bytes, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(tmp);
        if (e != hipSuccess) return device_fail(e, "amplitude copy");
        return PWA_OK;
    }
    if (is_mfma(m)) {   // the stored 16-bit amplitudes, widened to complex64
        const size_t bytes = (size_t)m->n * m->W * 8;
        void* tmp = nullptr;
        HIP_TRY(hipMalloc(&tmp, bytes));
        hipError_t e = pwa::launch_unpack_mfma(*m, (float*)tmp, s);
        if (e == hipSuccess) e = hipMemcpyAsync(out_host, tmp, bytes, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)hipFree(tmp);
        if (e != hipSuccess) return device_fail(e, "amplitude copy");
        return PWA_OK;
    }
    const bool c128 = m->form != pwa::kTable32;
    const size_t bytes = (size_t)m->n * m->P * (c128 ? 16 : 8);
    void* tmp = nullptr;
    HIP_TRY(hipMalloc(&tmp, bytes));
    hipError_t e;
    if (m->form == pwa::kTable64Plain)
        e = pwa::launch_unpack_soa((const double*)m->d_data, m->n, m->P, (double*)tmp, s);
    else
        e = pwa::launch_unpack_tiled(m->d_data, c128, m->n, m->W, m->d_pairs, tmp, s);
    if (e == hipSuccess) e = hipMemcpyAsync(out_host, tmp, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (e != hipSuccess) return device_fail(e, "table copy");
    return PWA_OK;
}

int pwa_copy_mc_matrix(const pwa_model* model, double* out_host, void* hip_stream)
{
    if (!model || !out_host) return fail(PWA_ERR_INVALID, "NULL model or out_host");
    const Model* m = reinterpret_cast<const Model*>(model);
    DeviceGuard g(m->device);
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_TRY(hipMemcpyAsync(out_host, m->d_M, sizeof(double) * 2 * m->W * m->W,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PWA_OK;
}

int pwa_set_mc_matrix(pwa_model* model, const double* m_host, void* hip_stream)
{
    if (!model || !m_host) return fail(PWA_ERR_INVALID, "NULL model or m_host");
    Model* m = reinterpret_cast<Model*>(model);
    for (int k = 0; k < 2 * m->W * m->W; ++k)
        if (!std::isfinite(m_host[k])) return fail(PWA_ERR_NONFINITE_INPUT, "M[%d] not finite", k / 2);
    DeviceGuard g(m->device);
    hipStream_t s = (hipStream_t)hip_stream;
    HIP_TRY(hipMemcpyAsync(m->d_M, m_host, sizeof(double) * 2 * m->W * m->W,
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return PWA_OK;
}

int pwa_get_amplitude_shape(const pwa_model* model, int32_t* lanes_per_event,
                            int32_t* waves_per_lane)
{
    if (!model || !lanes_per_event || !waves_per_lane) return fail(PWA_ERR_INVALID, "NULL argument");
    const Model* m = reinterpret_cast<const Model*>(model);
    if (m->form != pwa::kAmp32) return fail(PWA_ERR_INVALID, "not a PWA_FORM_AMPLITUDE model");
    *lanes_per_event = 1 << m->amp_lq;
    *waves_per_lane = m->amp_wl;
    return PWA_OK;
}

int pwa_set_amplitude_shape(pwa_model* model, int32_t lanes_per_event, int32_t waves_per_lane,
                            void* hip_stream)
{
    if (!model) return fail(PWA_ERR_INVALID, "NULL model");
    Model* m = reinterpret_cast<Model*>(model);
    if (m->form != pwa::kAmp32) return fail(PWA_ERR_INVALID, "not a PWA_FORM_AMPLITUDE model");
    if (!valid_shape(m->W, lanes_per_event, waves_per_lane))
        return fail(PWA_ERR_INVALID, "shape %d x %d does not hold %d waves (lanes 1..16, power of "
                    "two; waves per lane even, 2..16)", lanes_per_event, waves_per_lane, m->W);
    DeviceGuard g(m->device);
    return reshape_amp(m, pwa::AmpShape{log2_lanes(lanes_per_event), waves_per_lane},
                       (hipStream_t)hip_stream);
}

int pwa_tune_amplitude_shape(pwa_model* model, int32_t evals, void* hip_stream,
                             int32_t* lanes_per_event, int32_t* waves_per_lane)
{
    if (!model) return fail(PWA_ERR_INVALID, "NULL model");
    Model* m = reinterpret_cast<Model*>(model);
    if (m->form != pwa::kAmp32) return fail(PWA_ERR_INVALID, "not a PWA_FORM_AMPLITUDE model");
    if (evals < 1) return fail(PWA_ERR_INVALID, "evals must be >= 1");
    DeviceGuard g(m->device);
    hipStream_t s = (hipStream_t)hip_stream;
    // candidates: per lane count, the fewest even waves per lane that hold W,
    // if the row is at most a quarter longer than the shortest one
    std::vector<pwa::AmpShape> cand;
    int shortest = 1 << 30;
    for (int lq = 0; lq <= 4; ++lq) {
        int wl = (m->W + (1 << lq) - 1) >> lq;
        wl = std::max(2, wl + (wl & 1));
        if (wl <= pwa::kAmpMaxLaneWaves) shortest = std::min(shortest, wl << lq);
    }
    for (int lq = 0; lq <= 4; ++lq) {
        int wl = (m->W + (1 << lq) - 1) >> lq;
        wl = std::max(2, wl + (wl & 1));
        if (wl <= pwa::kAmpMaxLaneWaves && 4 * (wl << lq) <= 5 * shortest)
            cand.push_back(pwa::AmpShape{lq, wl});
    }
    pwa::VParams vp;
    std::memset(&vp, 0, sizeof vp);
    for (int a = 0; a < m->W; ++a) vp.v[2 * a] = 1.0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev()
        {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev_guard{e0, e1};
    // three passes over the candidates, keeping each one's fastest and slowest
    // time: the default shape stays unless a candidate's fastest time beats the
    // default's by more than the spread of either (a difference inside the
    // repeat-to-repeat spread decides nothing)
    const pwa::AmpShape def = pwa::amp_shape(m->W);
    std::vector<float> t_best(cand.size(), 0.f), t_worst(cand.size(), 0.f);
    for (int pass = 0; pass < 3; ++pass) {
        for (size_t c = 0; c < cand.size(); ++c) {
            int rc = reshape_amp(m, cand[c], s);
            if (rc != PWA_OK) return rc;
            HIP_TRY(pwa::launch_amp_fused(*m, vp, true, s, pwa::LaunchEvents{}));   // warm-up
            HIP_TRY(hipEventRecord(e0, s));
            for (int k = 0; k < evals; ++k)
                HIP_TRY(pwa::launch_amp_fused(*m, vp, true, s, pwa::LaunchEvents{}));
            HIP_TRY(hipEventRecord(e1, s));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (pass == 0 || ms < t_best[c]) t_best[c] = ms;
            if (pass == 0 || ms > t_worst[c]) t_worst[c] = ms;
        }
    }
    size_t d0 = cand.size();
    for (size_t c = 0; c < cand.size(); ++c)
        if (cand[c].lq == def.lq && cand[c].wl == def.wl) d0 = c;
    size_t bi = d0 < cand.size() ? d0 : 0;
    for (size_t c = 0; c < cand.size(); ++c) {
        const float margin = d0 < cand.size()
                                 ? std::max(t_worst[c] - t_best[c], t_worst[d0] - t_best[d0])
                                 : 0.f;
        if (c != bi && t_best[c] + margin < t_best[bi] &&
            (d0 >= cand.size() || t_best[c] + margin < t_best[d0]))
            bi = c;
    }
    const pwa::AmpShape best = cand[bi];
    const int rc = reshape_amp(m, best, s);
    if (rc != PWA_OK) return rc;
    if (lanes_per_event) *lanes_per_event = 1 << best.lq;
    if (waves_per_lane) *waves_per_lane = best.wl;
    return PWA_OK;
}

int pwa_set_timing(pwa_model* model, int enable)
{
    if (!model) return fail(PWA_ERR_INVALID, "NULL model");
    Model* m = reinterpret_cast<Model*>(model);
    if (enable && !m->ev_start[0]) {
        DeviceGuard g(m->device);
        for (int k = 0; k < Model::kTimingRing; ++k) {
            HIP_TRY(hipEventCreate(&m->ev_start[k]));
            HIP_TRY(hipEventCreate(&m->ev_stop[k]));
        }
    }
    if (enable < 0) return fail(PWA_ERR_INVALID, "enable must be >= 0");
    m->timing = enable;
    m->timing_count = 0;
    return PWA_OK;
}

int pwa_read_ceiling(const pwa_model* model, int32_t reps, void* hip_stream, double* ms,
                     int64_t* bytes)
{
    if (!model || !ms || !bytes) return fail(PWA_ERR_INVALID, "NULL model, ms or bytes");
    if (reps < 1) return fail(PWA_ERR_INVALID, "reps must be >= 1");
    const Model* m = reinterpret_cast<const Model*>(model);
    DeviceGuard g(m->device);
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t nbytes = m->data_bytes / 16 * 16;
    // the tiled tables: the fused kernel's own loads without its arithmetic;
    // other stored data: a plain reader of the same shape
    const bool tiled = m->form == pwa::kTable32 || m->form == pwa::kTable64Fused;
    const int sink_len = tiled ? m->grid * pwa::table_read_threads(*m) : 1024 * m->cus;
    uint32_t* sink = nullptr;
    HIP_TRY(hipMalloc(&sink, sizeof(uint32_t) * sink_len));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = -1.f;
    // one pass to warm up, then the fastest of reps timed passes
    for (int r = 0; r <= reps && e == hipSuccess; ++r) {
        e = tiled ? pwa::launch_table_read(*m, sink, s, pwa::LaunchEvents{e0, e1})
                  : pwa::launch_stream_read(m->d_data, nbytes, sink, sink_len, s,
                                            pwa::LaunchEvents{e0, e1});
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e == hipSuccess && r > 0 && (best < 0.f || t < best)) best = t;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    if (e != hipSuccess) return device_fail(e, "read-ceiling pass");
    *ms = best;
    *bytes = nbytes;
    return PWA_OK;
}

int pwa_build_timing(const pwa_model* model, double* table_ms, double* mc_ms)
{
    if (!model || !table_ms || !mc_ms) return fail(PWA_ERR_INVALID, "NULL argument");
    const Model* m = reinterpret_cast<const Model*>(model);
    *table_ms = m->build_table_ms;
    *mc_ms = m->build_mc_ms;
    return PWA_OK;
}

int pwa_get_timing(pwa_model* model, double* total_ms, int64_t* launches)
{
    if (!model || !total_ms || !launches) return fail(PWA_ERR_INVALID, "NULL argument");
    Model* m = reinterpret_cast<Model*>(model);
    if (m->ev_pending > 0) {
        DeviceGuard g(m->device);
        const int rc = read_timing(m, m->ev_pending);
        if (rc != PWA_OK) return rc;
    }
    *total_ms = m->timed_ms;
    *launches = m->timed_launches;
    m->timed_ms = 0.0;
    m->timed_launches = 0;
    return PWA_OK;
}

}  // extern "C"
