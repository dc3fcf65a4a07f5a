// C ABI of the p2o library: plan state, argument checks, memory carving and
// the launch sequences of each call.  See include/p2o.h for the contract.
#include "p2o.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"

using namespace p2o;

namespace {

thread_local std::string g_err;

p2o_status fail(p2o_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

enum PlanState { kCreated = 0, kBound = 1, kLoading = 2, kReady = 3 };

int64_t smooth7_at_least(int64_t n) {
    for (int64_t c = n < 1 ? 1 : n;; ++c) {
        int64_t m = c;
        for (int64_t p : {2, 3, 5, 7})
            while (m % p == 0) m /= p;
        if (m == 1) return c;
    }
}

bool have_device() {
    static bool found = false;        // a device, once seen, stays for the process
    if (found) return true;
    int n = 0;
    found = hipGetDeviceCount(&n) == hipSuccess && n > 0;
    if (!found) (void)hipGetLastError();
    return found;
}

}  // namespace

struct p2o_plan {
    int64_t Nd = 0, Nm = 0, Nt = 0, max_rhs = 0;
    int prec = 0;
    FftPlan fft{};
    int64_t L = 0, nfreq = 0, pitch = 0, nblk = 0;
    int elem_bytes = 0;        // stored complex entry
    int cbytes = 0;            // compute complex (16 FP64, 8 otherwise)
    int io_bytes = 0;          // element of m and d
    // spectrum store layout (bytes)
    size_t off_scales = 0, off_tw64 = 0, off_tw32 = 0, off_flag = 0, fhat_total = 0;
    // workspace layout (bytes), for max_rhs right-hand sides
    struct Carve {
        size_t off_X = 0, off_Y = 0, off_D = 0, off_P = 0, ws_total = 0;
        // FP16 matrix-core operands: wavefront maxima and right-hand-side scales of X and Y
        size_t off_A = 0, off_SX = 0, off_SY = 0;
        int amax_slots = 0;
        // online phase: a second data series buffer (I/O type) and FP64 data vectors
        size_t off_D2 = 0, off_Z = 0;
    } carve;
    size_t& off_X = carve.off_X;
    size_t& off_Y = carve.off_Y;
    size_t& off_D = carve.off_D;
    size_t& off_P = carve.off_P;
    size_t& ws_total = carve.ws_total;
    size_t& off_A = carve.off_A;
    size_t& off_SX = carve.off_SX;
    size_t& off_SY = carve.off_SY;
    int& amax_slots = carve.amax_slots;
    size_t& off_D2 = carve.off_D2;
    size_t& off_Z = carve.off_Z;
    // kernel configuration
    int fwd_rows = 64, fwd_nslab = 1, fwd_chunks = 1;
    int adj_rows = 1, adj_nslab = 1;
    int c2r_nd_blocks = 1;
    int batched_mode = P2O_BATCHED_AUTO;
    int gemm_tile = -1;                     // forced matrix-core tile variant, -1: tuned or built-in
    int qstride = 1;                        // data series observed every qstride-th step (multi-rate QoI maps)
    int fp16_ops = 1;                       // FP16 intermediate operands of F F* calls where possible
    std::map<int64_t, int> tuned_fwd, tuned_adj;   // autotuned variant per right-hand-side count
    // bound memory
    char* fhat = nullptr;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    int state = kCreated;
    bool aux_ready = false;
    std::vector<uint8_t> loaded;   // per column
    // per-stage timing
    bool prof = false;
    struct Rec { int stage; int64_t nrhs; hipEvent_t a, b; };
    int64_t cur_nrhs = 0;                               // right-hand sides of the call being enqueued
    std::map<std::pair<int, int64_t>, std::pair<double, int64_t>> by_nrhs;
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double tot_ms[P2O_STAGE_COUNT] = {};
    int64_t launches[P2O_STAGE_COUNT] = {};
    ~p2o_plan() {
        for (auto& r : pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

namespace {

p2o_status check_hip(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(P2O_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return P2O_OK;
}

hipEvent_t take_event(p2o_plan* p) {
    if (!p->pool.empty()) { hipEvent_t e = p->pool.back(); p->pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
    return e;
}

// Run one launcher; with profiling on, bracket it with events on the stream.
template <class Fn>
p2o_status staged(p2o_plan* p, int stage, const char* what, Fn&& launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (p->prof) {
        a = take_event(p);
        b = take_event(p);
        if (a && b) (void)hipEventRecord(a, p->stream);
    }
    const hipError_t e = launch();
    if (p->prof && a && b) {
        (void)hipEventRecord(b, p->stream);
        p->pending.push_back({stage, p->cur_nrhs, a, b});
    } else {
        if (a) p->pool.push_back(a);
        if (b) p->pool.push_back(b);
    }
    return check_hip(e, what);
}

p2o_status drain_profile(p2o_plan* p) {
    for (auto& r : p->pending) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return check_hip(e, "profile events");
        p->tot_ms[r.stage] += ms;
        p->launches[r.stage] += 1;
        auto& acc = p->by_nrhs[{r.stage, r.nrhs}];
        acc.first += ms;
        acc.second += 1;
        p->pool.push_back(r.a);
        p->pool.push_back(r.b);
    }
    p->pending.clear();
    return P2O_OK;
}

bool f64_plan(const p2o_plan* p) { return p->prec == kFP64; }
const void* tw_of(const p2o_plan* p) { return p->fhat + (f64_plan(p) ? p->off_tw64 : p->off_tw32); }
const float* scales_of(const p2o_plan* p) { return reinterpret_cast<const float*>(p->fhat + p->off_scales); }

// Spectrum columns that can be nonzero (Nm rounded up to 8); the rest of a
// row is zero padding that the products skip.
int64_t live_cols(const p2o_plan* p) { return (p->Nm + 7) / 8 * 8; }

void layout(p2o_plan* p) {
    const size_t nfreq = (size_t)p->nfreq;
    const size_t spec = nfreq * (size_t)p->Nd * (size_t)p->pitch * (size_t)p->elem_bytes;
    p->off_scales = align_up(spec);
    p->off_tw64 = align_up(p->off_scales + nfreq * (size_t)p->nblk * sizeof(float));
    p->off_tw32 = align_up(p->off_tw64 + (size_t)p->L * 16);
    p->off_flag = align_up(p->off_tw32 + (size_t)p->L * 8);
    p->fhat_total = align_up(p->off_flag + sizeof(unsigned));

    const size_t R = (size_t)p->max_rhs;
    const size_t xparts = (size_t)(p->adj_nslab > 1 ? p->adj_nslab : 1);
    size_t yparts = (size_t)(p->fwd_chunks > 1 ? p->fwd_chunks : 1);
    size_t ylen = yparts * nfreq * R * (size_t)p->Nd;
    if (p->prec == kBF16 || p->prec == kFP16) {
        // matrix-core path: forward partials per 4096-column chunk, and data
        // spectra in quad storage with rows padded to a multiple of 16
        ylen = std::max(ylen, (size_t)gemm_fwd_kchunks((int)live_cols(p)) * nfreq * R * (size_t)p->Nd);
        ylen = std::max(ylen, nfreq * R * (size_t)gemm_data_pitch((int)p->Nd));
    }
    p->off_X = 0;
    p->off_Y = align_up(p->off_X + xparts * nfreq * R * (size_t)p->pitch * p->cbytes);
    p->off_D = align_up(p->off_Y + ylen * p->cbytes);
    p->off_P = align_up(p->off_D + R * (size_t)p->Nt * (size_t)p->Nd * p->io_bytes);
    p->off_D2 = align_up(p->off_P + R * (size_t)p->c2r_nd_blocks * sizeof(double));
    p->off_Z = align_up(p->off_D2 + R * (size_t)p->Nt * (size_t)p->Nd * p->io_bytes);
    p->ws_total = align_up(p->off_Z + R * (size_t)p->Nt * (size_t)p->Nd * sizeof(double));
    if (p->prec == kFP16) {
        p->amax_slots = fft_amax_slots((int)std::max<int64_t>(p->pitch, gemm_data_pitch((int)p->Nd)));
        p->off_A = p->ws_total;
        // A: the transforms' amax partials, or a data-space column call's
        // FP16 operand scales (R) and row bounds (nfreq R)
        const size_t alen = std::max<size_t>((size_t)p->amax_slots, nfreq + 1);
        p->off_SX = align_up(p->off_A + R * alen * sizeof(float));
        p->off_SY = align_up(p->off_SX + R * sizeof(float));
        p->ws_total = align_up(p->off_SY + R * sizeof(float));
    }
}

p2o_status ready_for_apply(const p2o_plan* p, const void* a, const void* b, int64_t nrhs) {
    if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
    if (!a || !b) return fail(P2O_ERR_ARG, "input or output pointer is NULL");
    if (nrhs < 1 || nrhs > p->max_rhs)
        return fail(P2O_ERR_ARG, "nrhs=%lld outside [1, max_rhs=%lld]", (long long)nrhs, (long long)p->max_rhs);
    if (p->state != kReady) return fail(P2O_ERR_STATE, "spectrum not loaded (call p2o_load_blocks and p2o_load_finalize)");
    if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
    return P2O_OK;
}

// descriptors --------------------------------------------------------------
// parameter-side series: time [b][t][Nm]  <->  spectrum [w][b][pitch] (+ partials)
SeriesIO io_param(const p2o_plan* p, int64_t nrhs, const int32_t* nt_active, int nparts) {
    SeriesIO io{};
    io.t_stride = p->Nm;
    io.t_outer = p->Nt * p->Nm;
    io.f_stride = nrhs * p->pitch;
    io.f_outer = p->pitch;
    io.f_part = p->nfreq * nrhs * p->pitch;
    io.nparts = nparts;
    io.S = (int)p->Nm;
    io.S_pad = (int)p->pitch;
    io.Nt = (int)p->Nt;
    io.outer_count = (int)nrhs;
    io.nt_active = nt_active;
    return io;
}

// data-side series: time [b][t][Nd]  <->  spectrum [w][b][Nd] (+ partials)
SeriesIO io_data(const p2o_plan* p, int64_t nrhs, const int32_t* nt_active, int nparts) {
    SeriesIO io{};
    io.t_stride = p->Nd;
    io.t_outer = p->Nt * p->Nd;
    io.f_stride = nrhs * p->Nd;
    io.f_outer = p->Nd;
    io.f_part = p->nfreq * nrhs * p->Nd;
    io.nparts = nparts;
    io.S = (int)p->Nd;
    io.S_pad = (int)p->Nd;
    io.Nt = (int)p->Nt;
    io.outer_count = (int)nrhs;
    io.nt_active = nt_active;
    return io;
}

GemvArgs gemv_args(const p2o_plan* p, int64_t nrhs, bool fwd) {
    GemvArgs ga{};
    ga.Nd = (int)p->Nd;
    ga.pitch = (int)p->pitch;
    ga.ncols = (int)live_cols(p);
    ga.nfreq = (int)p->nfreq;
    ga.nrhs = (int)nrhs;
    ga.nblk = (int)p->nblk;
    ga.nslab = fwd ? p->fwd_nslab : p->adj_nslab;
    ga.rows_per_wg = fwd ? p->fwd_rows : p->adj_rows;
    ga.part_stride = fwd ? p->nfreq * nrhs * p->Nd : p->nfreq * nrhs * p->pitch;
    return ga;
}

// enqueue sequences ----------------------------------------------------------
// Several right-hand sides with a BF16 (or FP16, on the LDS-ring kernels,
// for shapes they can address) spectrum go to the matrix cores.  Their
// operands are written by the FFTs in quad storage, in place by the F F*
// projection, whose tiles must then span whole groups of 4 series.
bool mfma_capable(const p2o_plan* p) {
    return p->prec == kBF16 || (p->prec == kFP16 && gemm_f16_fits((int)p->Nd, (int)p->pitch));
}

bool mfma_on(const p2o_plan* p, int64_t nrhs) {
    if (!mfma_capable(p)) return false;
    if (fft_tile_shift(p->fft.M, false) < 2) return false;
    if (p->batched_mode == P2O_BATCHED_MFMA) return true;
    if (p->batched_mode == P2O_BATCHED_GEMV) return false;
    return nrhs >= 2;
}

int fwd_parts(const p2o_plan* p, int64_t nrhs) {
    return mfma_on(p, nrhs) ? gemm_fwd_kchunks((int)live_cols(p)) : p->fwd_chunks;
}

int adj_parts(const p2o_plan* p, int64_t nrhs) { return mfma_on(p, nrhs) ? 1 : p->adj_nslab; }

GemmArgs gemm_args(const p2o_plan* p, int64_t nrhs) {
    GemmArgs ga{};
    ga.Nd = (int)p->Nd;
    ga.pitch = (int)p->pitch;
    ga.ncols = (int)live_cols(p);
    ga.nfreq = (int)p->nfreq;
    ga.nrhs = (int)nrhs;
    ga.nblk = (int)p->nblk;
    ga.part_stride = p->nfreq * nrhs * p->Nd;
    ga.a_f16 = p->prec == kFP16;
    ga.rhs_scale = nullptr;
    return ga;
}

float* scale_X(const p2o_plan* p) { return reinterpret_cast<float*>(p->ws + p->off_SX); }
float* scale_Y(const p2o_plan* p) { return reinterpret_cast<float*>(p->ws + p->off_SY); }

// Operands of the matrix-core products written by a transform: quad BF16
// hi/lo for a BF16 spectrum; complex FP32 with wavefront maxima and
// per-right-hand-side scales (into `scale`) for an FP16 spectrum.
void rhs_operand(const p2o_plan* p, int64_t nrhs, SeriesIO& io, float* scale) {
    if (!mfma_on(p, nrhs)) return;
    if (p->prec == kFP16) {
        io.quad = 0;
        io.amax_part = reinterpret_cast<float*>(p->ws + p->off_A);
        io.amax_slots = p->amax_slots;
        io.rhs_scale = scale;
    } else {
        io.quad = 1;
    }
}

// matrix-core tile variant for a call with nrhs right-hand sides
int gemm_tile_for(const p2o_plan* p, const std::map<int64_t, int>& tuned, int64_t nrhs) {
    if (p->gemm_tile >= 0) return p->gemm_tile;
    auto it = tuned.find(nrhs);
    return it == tuned.end() ? -1 : it->second;
}

// X (parameter spectra) -> Y partial products; xscale: the FP16 operand
// scales written with X (this plan's own unless X comes from another plan)
p2o_status enqueue_fwd_products(p2o_plan* p, const void* X, void* Y, int64_t nrhs, const float* xscale = nullptr) {
    if (mfma_on(p, nrhs))
        return staged(p, P2O_STAGE_GEMM_FWD, "forward per-frequency products (matrix cores)", [&] {
            GemmArgs ga = gemm_args(p, nrhs);
            ga.rhs_scale = xscale ? xscale : scale_X(p);
            return launch_gemm_fwd(ga, gemm_tile_for(p, p->tuned_fwd, nrhs), p->fhat, scales_of(p), X, Y, p->stream);
        });
    return staged(p, P2O_STAGE_GEMV_FWD, "forward per-frequency products", [&] {
        return launch_gemv_fwd(p->prec, gemv_args(p, nrhs, true), p->fhat, scales_of(p), X, Y, p->stream);
    });
}

// Y (data spectra) -> X partial products
p2o_status enqueue_adj_products(p2o_plan* p, const void* Y, void* X, int64_t nrhs) {
    if (mfma_on(p, nrhs))
        return staged(p, P2O_STAGE_GEMM_ADJ, "adjoint per-frequency products (matrix cores)", [&] {
            GemmArgs ga = gemm_args(p, nrhs);
            ga.rhs_scale = scale_Y(p);
            return launch_gemm_adj(ga, gemm_tile_for(p, p->tuned_adj, nrhs), p->fhat, scales_of(p), Y, X, p->stream);
        });
    return staged(p, P2O_STAGE_GEMV_ADJ, "adjoint per-frequency products", [&] {
        return launch_gemv_adj(p->prec, gemv_args(p, nrhs, false), p->fhat, scales_of(p), Y, X, p->stream);
    });
}

// parameter spectra for the forward products (matrix-core operand form on
// that path)
SeriesIO io_param_rhs(const p2o_plan* p, int64_t nrhs, const int32_t* nt_active, int nparts) {
    SeriesIO io = io_param(p, nrhs, nt_active, nparts);
    rhs_operand(p, nrhs, io, scale_X(p));
    return io;
}

// data spectra for the adjoint products: on the matrix-core path in operand
// form, rows padded with zeros to gemm_data_pitch(Nd)
SeriesIO io_data_rhs(const p2o_plan* p, int64_t nrhs, const int32_t* nt_active) {
    SeriesIO io = io_data(p, nrhs, nt_active, 1);
    if (mfma_on(p, nrhs)) {
        const int ld = gemm_data_pitch((int)p->Nd);
        io.f_stride = nrhs * ld;
        io.f_outer = ld;
        io.f_part = p->nfreq * nrhs * ld;
        io.S_pad = ld;
        rhs_operand(p, nrhs, io, scale_Y(p));
    }
    return io;
}

p2o_status enqueue_forward_to_Y(p2o_plan* p, const void* m, int64_t nrhs, const int32_t* nt) {
    void* X = p->ws + p->off_X;
    void* Y = p->ws + p->off_Y;
    p2o_status s = staged(p, P2O_STAGE_R2C, "r2c (parameters)", [&] {
        return launch_r2c(f64_plan(p), f64_plan(p), p->fft, io_param_rhs(p, nrhs, nt, 1), m, X, tw_of(p), p->stream);
    });
    if (s) return s;
    return enqueue_fwd_products(p, X, Y, nrhs);
}

p2o_status enqueue_adjoint_to_X(p2o_plan* p, const void* d, int64_t nrhs, const int32_t* nt) {
    void* X = p->ws + p->off_X;
    void* Y = p->ws + p->off_Y;
    p2o_status s = staged(p, P2O_STAGE_R2C, "r2c (data)", [&] {
        return launch_r2c(f64_plan(p), f64_plan(p), p->fft, io_data_rhs(p, nrhs, nt), d, Y, tw_of(p), p->stream);
    });
    if (s) return s;
    return enqueue_adj_products(p, Y, X, nrhs);
}

p2o_status noise_mode(const p2o_plan* p, int64_t len, int* mode) {
    if (len == 1) *mode = 0;
    else if (len == p->Nd) *mode = 1;
    else if (len == p->Nd * p->Nt) *mode = 2;
    else
        return fail(P2O_ERR_ARG, "noise_var_len=%lld must be 1, Nd=%lld or Nt*Nd=%lld", (long long)len,
                    (long long)p->Nd, (long long)(p->Nd * p->Nt));
    return P2O_OK;
}

p2o_status enqueue_apply_Ft(p2o_plan* p, const void* d, void* m, int64_t nrhs, const int32_t* nt_active) {
    p->cur_nrhs = nrhs;
    p2o_status s = enqueue_adjoint_to_X(p, d, nrhs, nt_active);
    if (s) return s;
    return staged(p, P2O_STAGE_C2R, "c2r (parameters)", [&] {
        return launch_c2r(f64_plan(p), p->fft, io_param(p, nrhs, nt_active, adj_parts(p, nrhs)), p->ws + p->off_X, m,
                          tw_of(p), nullptr, nullptr, 0, nullptr, p->stream);
    });
}

// The FP16-operand form of an F F* call is possible: FP16 spectrum on the
// matrix cores, one adjoint partial and a compiled-length re-pad for the
// shape (the forward products take the whole-line ring: 64- or 128-row tiles
// for at most 64 or 128 sensors, 320-row ones above).
bool fp16_operands_ok(const p2o_plan* p, int64_t nrhs, const int32_t* nt_active) {
    if (!p->fp16_ops || p->prec != kFP16 || !mfma_on(p, nrhs) || adj_parts(p, nrhs) != 1) return false;
    return launch_project_half(p->fft, io_param(p, nrhs, nt_active, 1), nullptr, nullptr, nullptr, nullptr, nullptr,
                               nullptr);
}

// F G* with FP16 intermediate operands (F G* = F F* when F and G are the
// same plan): G's data-side r2c and the operand scales (bounded from the data
// spectra and G's block multipliers), G's adjoint products written as scaled
// FP16 pairs into G's X, the re-pad in place on them, F's forward products
// reading them as FP16 right-hand sides, F's data-side c2r.  sx lives in G's
// wavefront-maximum region (free once the data-side scales are taken), sy in
// G's parameter-side scales.
p2o_status enqueue_cross_half(p2o_plan* F, p2o_plan* G, const void* e, void* h, int64_t nrhs,
                              const int32_t* nt_active) {
    void* X = G->ws + G->off_X;
    void* YG = G->ws + G->off_Y;
    void* YF = F->ws + F->off_Y;
    float* sx = reinterpret_cast<float*>(G->ws + G->off_A);
    float* sy = scale_X(G);
    const int ld = gemm_data_pitch((int)G->Nd);
    p2o_status s = staged(G, P2O_STAGE_R2C, "r2c (data) and FP16 operand scales", [&] {
        hipError_t err = launch_r2c(false, false, G->fft, io_data_rhs(G, nrhs, nt_active), e, YG, tw_of(G), G->stream);
        if (err != hipSuccess) return err;
        return launch_fp16_operand_scales(YG, ld, (int)nrhs, (int)G->nfreq, (int)G->Nd, scales_of(G), (int)G->nblk,
                                          (int)G->Nt, sx + G->max_rhs, sx, sy, G->stream);
    });
    if (s) return s;
    s = staged(G, P2O_STAGE_GEMM_ADJ, "adjoint per-frequency products (matrix cores, FP16 out)", [&] {
        GemmArgs ga = gemm_args(G, nrhs);
        ga.rhs_scale = scale_Y(G);
        ga.out_scale = sx;
        return launch_gemm_adj(ga, gemm_tile_for(G, G->tuned_adj, nrhs), G->fhat, scales_of(G), YG, X, G->stream);
    });
    if (s) return s;
    s = staged(G, P2O_STAGE_PROJECT, "truncate and re-pad (FP16 operands)", [&] {
        hipError_t err = hipErrorInvalidValue;
        if (!launch_project_half(G->fft, io_param(G, nrhs, nt_active, 1), X, tw_of(G), sx, sy, G->stream, &err))
            return hipErrorInvalidValue;
        return err;
    });
    if (s) return s;
    s = staged(F, P2O_STAGE_GEMM_FWD, "forward per-frequency products (matrix cores, FP16 operands)", [&] {
        GemmArgs ga = gemm_args(F, nrhs);
        ga.rhs_scale = sy;
        ga.b_f16 = 1;                                     // the whole-line tile for F's sensor count
        return launch_gemm_fwd(ga, -1, F->fhat, scales_of(F), X, YF, F->stream);
    });
    if (s) return s;
    return staged(F, P2O_STAGE_C2R, "c2r (data)", [&] {
        return launch_c2r(false, F->fft, io_data(F, nrhs, nt_active, fwd_parts(F, nrhs)), YF, h, tw_of(F), nullptr,
                          nullptr, 0, nullptr, F->stream);
    });
}

p2o_status enqueue_FFt(p2o_plan* p, const void* e, void* h, int64_t nrhs, const int32_t* nt_active) {
    p->cur_nrhs = nrhs;
    if (fp16_operands_ok(p, nrhs, nt_active)) return enqueue_cross_half(p, p, e, h, nrhs, nt_active);
    p2o_status s = enqueue_adjoint_to_X(p, e, nrhs, nt_active);
    if (s) return s;
    s = staged(p, P2O_STAGE_PROJECT, "truncate and re-pad", [&] {
        return launch_project(f64_plan(p), p->fft, io_param_rhs(p, nrhs, nt_active, adj_parts(p, nrhs)),
                              p->ws + p->off_X, tw_of(p), p->stream);
    });
    if (s) return s;
    s = enqueue_fwd_products(p, p->ws + p->off_X, p->ws + p->off_Y, nrhs);
    if (s) return s;
    return staged(p, P2O_STAGE_C2R, "c2r (data)", [&] {
        return launch_c2r(f64_plan(p), p->fft, io_data(p, nrhs, nt_active, fwd_parts(p, nrhs)), p->ws + p->off_Y, h,
                          tw_of(p), nullptr, nullptr, 0, nullptr, p->stream);
    });
}

p2o_status enqueue_apply_F(p2o_plan* p, const void* m, void* d, int64_t nrhs, const int32_t* nt_active) {
    p->cur_nrhs = nrhs;
    p2o_status s = enqueue_forward_to_Y(p, m, nrhs, nt_active);
    if (s) return s;
    return staged(p, P2O_STAGE_C2R, "c2r (data)", [&] {
        return launch_c2r(f64_plan(p), p->fft, io_data(p, nrhs, nt_active, fwd_parts(p, nrhs)), p->ws + p->off_Y, d,
                          tw_of(p), nullptr, nullptr, 0, nullptr, p->stream);
    });
}

// h = F G^* e for two plans with the same parameter grid (Nm, Nt) and
// storage: G's adjoint pass and the truncate-and-re-pad in G's workspace,
// then F's forward products on G's parameter spectra and F's inverse FFT.
// e and h are full-grid series (every step).
p2o_status enqueue_cross(p2o_plan* F, p2o_plan* G, const void* e, void* h, int64_t nrhs) {
    G->cur_nrhs = nrhs;
    F->cur_nrhs = nrhs;
    if (fp16_operands_ok(G, nrhs, nullptr) && F->fp16_ops && F->prec == kFP16 && mfma_on(F, nrhs))
        return enqueue_cross_half(F, G, e, h, nrhs, nullptr);
    p2o_status s = enqueue_adjoint_to_X(G, e, nrhs, nullptr);
    if (s) return s;
    s = staged(G, P2O_STAGE_PROJECT, "truncate and re-pad", [&] {
        return launch_project(f64_plan(G), G->fft, io_param_rhs(G, nrhs, nullptr, adj_parts(G, nrhs)),
                              G->ws + G->off_X, tw_of(G), G->stream);
    });
    if (s) return s;
    s = enqueue_fwd_products(F, G->ws + G->off_X, F->ws + F->off_Y, nrhs, scale_X(G));
    if (s) return s;
    return staged(F, P2O_STAGE_C2R, "c2r (data)", [&] {
        return launch_c2r(f64_plan(F), F->fft, io_data(F, nrhs, nullptr, fwd_parts(F, nrhs)), F->ws + F->off_Y, h,
                          tw_of(F), nullptr, nullptr, 0, nullptr, F->stream);
    });
}

// Multi-rate plans exchange data series of Nt / qstride steps: expand one
// to the full grid (zeros between its steps) in `full`, or sample a full one.
p2o_status qoi_expand(p2o_plan* p, const void* q, void* full, int64_t nrhs) {
    return check_hip(launch_qoi_scatter(f64_plan(p), q, full, (int)p->Nt, (int)p->Nd, p->qstride, (int)nrhs, p->stream),
                     "series to the full grid");
}
p2o_status qoi_sample(p2o_plan* p, const void* full, void* q, int64_t nrhs) {
    return check_hip(launch_qoi_gather(f64_plan(p), full, q, nullptr, 0, 0, 1.0, false, (int)p->Nt, (int)p->Nd,
                                       p->qstride, (int)nrhs, p->stream), "series at the observed steps");
}

p2o_status every_step(const p2o_plan* p, const char* what) {
    if (p->qstride != 1)
        return fail(P2O_ERR_STATE, "%s needs data at every step (the plan observes every %d-th step)", what, p->qstride);
    return P2O_OK;
}

// Two plans that share the parameter grid, storage and stream, ready for
// nrhs right-hand sides.
p2o_status compatible(const p2o_plan* F, const p2o_plan* G, int64_t nrhs) {
    if (!F || !G) return fail(P2O_ERR_ARG, "plan is NULL");
    if (F->Nm != G->Nm || F->Nt != G->Nt)
        return fail(P2O_ERR_ARG, "plans differ in Nm (%lld, %lld) or Nt (%lld, %lld)", (long long)F->Nm,
                    (long long)G->Nm, (long long)F->Nt, (long long)G->Nt);
    if (F->prec != G->prec) return fail(P2O_ERR_DTYPE, "plans differ in storage precision");
    if (F->stream != G->stream) return fail(P2O_ERR_ARG, "plans must use the same stream");
    if (F->state != kReady || G->state != kReady)
        return fail(P2O_ERR_STATE, "spectrum not loaded (call p2o_load_blocks and p2o_load_finalize)");
    if (nrhs < 1 || nrhs > F->max_rhs || nrhs > G->max_rhs)
        return fail(P2O_ERR_ARG, "nrhs=%lld outside [1, min(max_rhs)=%lld]", (long long)nrhs,
                    (long long)std::min(F->max_rhs, G->max_rhs));
    if (mfma_on(F, nrhs) != mfma_on(G, nrhs))
        return fail(P2O_ERR_STATE, "the plans take different product paths for %lld right-hand sides (batched modes)",
                    (long long)nrhs);
    if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
    return P2O_OK;
}

// ---------------------------------------------------------------- scratch of the allocation-free entry point
// p2o_apply_F_noalloc's workspace: a fixed array in device memory (each GPU
// the library runs on holds its own copy until the process ends).  Host code
// never uses the array's name as an address: its device address, taken once
// per device with hipGetSymbolAddress while that device is current, is kept
// in g_scratch and used for every access.  Every call on a device shares
// that device's array: calls that overlap on one GPU race.  Nothing in it
// needs to start at zero (the transforms and products write every value
// they later read).
constexpr size_t kScratchBytes = size_t(128) << 20;
__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch;

p2o_status scratch_on_current_device(const p2o_plan* p, void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(P2O_ERR_HIP, "hipGetDevice failed");
    }
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p->fhat) != hipSuccess) {
        (void)hipGetLastError();
        return fail(P2O_ERR_HIP, "cannot query the spectrum's device");
    }
    if (at.device != dev)
        return fail(P2O_ERR_ARG, "the plan's spectrum is on device %d but device %d is current", at.device, dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        *out = it->second;
        return P2O_OK;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(P2O_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    }
    g_scratch[dev] = ptr;
    *out = ptr;
    return P2O_OK;
}

}  // namespace

// ============================================================================
extern "C" {

const char* p2o_status_string(int32_t st) {
    switch (st) {
        case P2O_OK: return "P2O_OK";
        case P2O_ERR_ARG: return "P2O_ERR_ARG";
        case P2O_ERR_STATE: return "P2O_ERR_STATE";
        case P2O_ERR_DTYPE: return "P2O_ERR_DTYPE";
        case P2O_ERR_STORAGE: return "P2O_ERR_STORAGE";
        case P2O_ERR_NONFINITE: return "P2O_ERR_NONFINITE";
        case P2O_ERR_HIP: return "P2O_ERR_HIP";
        case P2O_ERR_NO_DEVICE: return "P2O_ERR_NO_DEVICE";
        default: return "P2O_UNKNOWN_STATUS";
    }
}

const char* p2o_last_error(void) { return g_err.c_str(); }

p2o_status p2o_create(p2o_plan** out, int64_t Nd, int64_t Nm, int64_t Nt, int32_t precision, int64_t max_rhs) {
    try {
        if (!out) return fail(P2O_ERR_ARG, "out is NULL");
        if (Nd < 1 || Nm < 1 || Nt < 1)
            return fail(P2O_ERR_ARG, "shape Nd=%lld Nm=%lld Nt=%lld must be positive", (long long)Nd, (long long)Nm,
                        (long long)Nt);
        if (max_rhs < 1 || max_rhs > 65535) return fail(P2O_ERR_ARG, "max_rhs=%lld outside [1, 65535]", (long long)max_rhs);
        if (precision < P2O_FP64 || precision > P2O_FP16)
            return fail(P2O_ERR_DTYPE, "unknown precision %d", (int)precision);
        if (Nd > (1 << 24) || Nm > (1LL << 30))
            return fail(P2O_ERR_ARG, "Nd=%lld or Nm=%lld too large", (long long)Nd, (long long)Nm);
        const int64_t M = smooth7_at_least(Nt);
        FftPlan fp{};
        fp.M = (int)M;
        fp.L = (int)(2 * M);
        int64_t m = M;
        int np = 0;
        for (int r : {8, 4, 2, 3, 5, 7})
            while (m % r == 0 && np < kMaxPasses) { fp.radix[np++] = r; m /= r; }
        fp.npass = np;
        fp.fixed = 1;
        if (m != 1 || fft_tile_shift((int)M, true) < 0 || fft_tile_shift((int)M, false) < 0 || load_tile_shift((int)M) < 0)
            return fail(P2O_ERR_ARG, "Nt=%lld too long (transform length %lld exceeds the LDS tile)", (long long)Nt,
                        (long long)(2 * M));

        p2o_plan* p = new (std::nothrow) p2o_plan();
        if (!p) return fail(P2O_ERR_ARG, "out of host memory");
        p->Nd = Nd; p->Nm = Nm; p->Nt = Nt; p->max_rhs = max_rhs; p->prec = precision;
        p->fft = fp;
        p->L = 2 * M;
        p->nfreq = M + 1;
        // Rows start an odd number of 128-byte lines apart (pitch = 32 mod 64
        // entries): with a power-of-two pitch every row of a tile maps to the
        // same L2 sets, and rows read a part of a line at a time lose their
        // lines before the rest is read.
        p->pitch = (Nm + 31) / 64 * 64 + 32;
        p->nblk = (Nm + kScaleBlock - 1) / kScaleBlock;
        p->elem_bytes = precision == P2O_FP64 ? 16 : precision == P2O_FP32 ? 8 : 4;
        p->cbytes = precision == P2O_FP64 ? 16 : 8;
        p->io_bytes = precision == P2O_FP64 ? 8 : 4;
        p->fwd_rows = 64;
        p->fwd_nslab = (int)((Nd + p->fwd_rows - 1) / p->fwd_rows);
        p->fwd_chunks = gemv_fwd_chunks(precision, (int)((Nm + 7) / 8 * 8));
        p->adj_nslab = 1;
        p->adj_rows = (int)Nd;
        p->c2r_nd_blocks = c2r_grid_x(fp, precision == P2O_FP64, (int)Nd);
        layout(p);
        p->loaded.assign((size_t)Nm, 0);
        *out = p;
        return P2O_OK;
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_create");
    }
}

p2o_status p2o_bandwidth_probe(int32_t mode, const void* src, void* dst, size_t bytes, int32_t blocks,
                               void* stream) {
    if (mode != 0 && mode != 1) return fail(P2O_ERR_ARG, "probe mode must be 0 (read) or 1 (copy)");
    if (!src || !dst) return fail(P2O_ERR_ARG, "probe buffer is NULL");
    if (bytes == 0 || bytes % (mode == 0 ? 2048 : 32))
        return fail(P2O_ERR_ARG, "probe size must be a positive multiple of %d", mode == 0 ? 2048 : 32);
    if (blocks < 1 || blocks > 65536) return fail(P2O_ERR_ARG, "probe blocks must be in [1, 65536]");
    if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 32)
        return fail(P2O_ERR_ARG, "probe buffers must be 32-byte aligned");
    if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
    return check_hip(launch_probe(mode, src, dst, bytes, blocks, static_cast<hipStream_t>(stream)), "bandwidth probe");
}

p2o_status p2o_set_option(p2o_plan* p, int32_t option, int64_t value) {
    if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
    if (option == P2O_OPT_BATCHED) {
        if (value < P2O_BATCHED_AUTO || value > P2O_BATCHED_MFMA)
            return fail(P2O_ERR_ARG, "batched mode %lld unknown", (long long)value);
        if (value == P2O_BATCHED_MFMA && !mfma_capable(p))
            return fail(P2O_ERR_DTYPE, "the matrix-core path needs a BF16 or FP16 spectrum");
        p->batched_mode = (int)value;
        return P2O_OK;
    }
    if (option == P2O_OPT_GEMM_TILE) {
        if (value < -1 || value >= gemm_tile_count())
            return fail(P2O_ERR_ARG, "tile variant %lld not in [-1, %d)", (long long)value, gemm_tile_count());
        p->gemm_tile = (int)value;
        return P2O_OK;
    }
    if (option == P2O_OPT_FFT_FIXED) {
        if (value != 0 && value != 1) return fail(P2O_ERR_ARG, "fixed-length FFT switch %lld is not 0 or 1", (long long)value);
        p->fft.fixed = (int)value;
        return P2O_OK;
    }
    if (option == P2O_OPT_FP16_OPERANDS) {
        if (value != 0 && value != 1) return fail(P2O_ERR_ARG, "FP16 operand switch %lld is not 0 or 1", (long long)value);
        p->fp16_ops = (int)value;
        return P2O_OK;
    }
    if (option == P2O_OPT_OUTPUT_STRIDE) {
        if (value < 1 || value > p->Nt || p->Nt % value != 0)
            return fail(P2O_ERR_ARG, "output stride %lld must divide Nt=%lld", (long long)value, (long long)p->Nt);
        p->qstride = (int)value;
        return P2O_OK;
    }
    return fail(P2O_ERR_ARG, "unknown option %d", (int)option);
}

p2o_status p2o_gemm_tile_info(int32_t tile, int32_t* row_groups, int32_t* substeps, int32_t* blocks,
                              int32_t* rhs_per_group) {
    int rg = 0, ku = 0, mb = 0, nr = 0;
    if (gemm_tile_shape(tile, &rg, &ku, &mb, &nr))
        return fail(P2O_ERR_ARG, "tile variant %d not in [0, %d)", (int)tile, gemm_tile_count());
    if (row_groups) *row_groups = rg;
    if (substeps) *substeps = ku;
    if (blocks) *blocks = mb;
    if (rhs_per_group) *rhs_per_group = nr;
    return P2O_OK;
}

p2o_status p2o_autotune(p2o_plan* p, int64_t nrhs, int32_t reps, int32_t* fwd_tile, int32_t* adj_tile,
                        double* fwd_ms, double* adj_ms) {
    try {
        if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
        if (p->state != kReady) return fail(P2O_ERR_STATE, "spectrum not loaded (call p2o_load_blocks and p2o_load_finalize)");
        if (nrhs < 1 || nrhs > p->max_rhs) return fail(P2O_ERR_ARG, "nrhs=%lld not in [1, %lld]", (long long)nrhs, (long long)p->max_rhs);
        if (reps < 1 || reps > 100) return fail(P2O_ERR_ARG, "reps=%d not in [1, 100]", (int)reps);
        if (!mfma_on(p, nrhs)) return fail(P2O_ERR_DTYPE, "calls with nrhs=%lld do not use the matrix cores on this plan", (long long)nrhs);
        if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
        // Operands: the workspace's spectra regions, filled with finite random
        // BF16 words (on zeros the matrix cores run cooler and faster than on
        // real data, which would skew the comparison).  The adjoint's operand
        // is refilled after the forward launches have written over it.
        void* X = p->ws + p->off_X;
        void* Y = p->ws + p->off_Y;
        p2o_status s = check_hip(launch_fill_bf16(X, p->off_D - p->off_X, 0x5EEDu, p->stream), "autotune operand fill");
        if (s) return s;
        if (p->prec == kFP16) {
            // FP16 plans read the operands as complex FP32 (the words above are
            // finite, magnitudes in [1/2, 1)) with unit right-hand-side scales
            s = check_hip(launch_fill_f32(scale_X(p), (size_t)p->max_rhs, 1.f, p->stream), "autotune scale fill");
            if (!s) s = check_hip(launch_fill_f32(scale_Y(p), (size_t)p->max_rhs, 1.f, p->stream), "autotune scale fill");
            if (s) return s;
        }
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            if (a) (void)hipEventDestroy(a);
            return fail(P2O_ERR_HIP, "event creation failed");
        }
        GemmArgs gf = gemm_args(p, nrhs), gb = gemm_args(p, nrhs);
        gf.rhs_scale = scale_X(p);                      // the forward reads X, the adjoint Y
        gb.rhs_scale = scale_Y(p);
        const bool a_f16 = gf.a_f16 != 0;
        double best[2] = {1e300, 1e300};
        int pick[2] = {-1, -1};
        for (int dir = 0; dir < 2 && !s; ++dir) {
            if (dir == 1) s = check_hip(launch_fill_bf16(Y, p->off_D - p->off_Y, 0xADu, p->stream), "autotune operand fill");
            for (int t = 0; t < gemm_tile_count() && !s; ++t) {
                if (!gemm_tile_has(t, dir == 0) || (a_f16 && !gemm_tile_is_ring(t))) continue;
                auto run = [&]() {
                    return dir == 0 ? launch_gemm_fwd(gf, t, p->fhat, scales_of(p), X, Y, p->stream)
                                    : launch_gemm_adj(gb, t, p->fhat, scales_of(p), Y, X, p->stream);
                };
                s = check_hip(run(), "autotune warm-up launch");
                if (s) break;
                s = check_hip(hipEventRecord(a, p->stream), "event record");
                for (int r = 0; r < reps && !s; ++r) s = check_hip(run(), "autotune launch");
                if (!s) s = check_hip(hipEventRecord(b, p->stream), "event record");
                if (!s) s = check_hip(hipEventSynchronize(b), "autotune synchronisation");
                float ms = 0.f;
                if (!s) s = check_hip(hipEventElapsedTime(&ms, a, b), "event timing");
                if (!s && ms / reps < best[dir]) { best[dir] = ms / reps; pick[dir] = t; }
            }
        }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        if (s) return s;
        p->tuned_fwd[nrhs] = pick[0];
        p->tuned_adj[nrhs] = pick[1];
        if (fwd_tile) *fwd_tile = pick[0];
        if (adj_tile) *adj_tile = pick[1];
        if (fwd_ms) *fwd_ms = best[0];
        if (adj_ms) *adj_ms = best[1];
        return P2O_OK;
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_autotune");
    }
}

p2o_status p2o_profile_enable(p2o_plan* p, int32_t enable) {
    if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
    if (enable != 0 && enable != 1) return fail(P2O_ERR_ARG, "enable must be 0 or 1");
    if (!p->pending.empty()) {
        if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
        p2o_status s = drain_profile(p);
        if (s) return s;
    }
    for (int i = 0; i < P2O_STAGE_COUNT; ++i) { p->tot_ms[i] = 0.0; p->launches[i] = 0; }
    p->by_nrhs.clear();
    p->prof = enable != 0;
    return P2O_OK;
}

p2o_status p2o_profile_read(p2o_plan* p, int32_t stage, double* total_ms, int64_t* launches) {
    if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
    if (stage < 0 || stage >= P2O_STAGE_COUNT) return fail(P2O_ERR_ARG, "unknown stage %d", (int)stage);
    if (!total_ms && !launches) return fail(P2O_ERR_ARG, "both outputs are NULL");
    if (!p->pending.empty()) {
        if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
        p2o_status s = drain_profile(p);
        if (s) return s;
    }
    if (total_ms) *total_ms = p->tot_ms[stage];
    if (launches) *launches = p->launches[stage];
    return P2O_OK;
}

p2o_status p2o_profile_read_nrhs(p2o_plan* p, int32_t stage, int64_t nrhs, double* total_ms, int64_t* launches) {
    if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
    if (stage < 0 || stage >= P2O_STAGE_COUNT) return fail(P2O_ERR_ARG, "unknown stage %d", (int)stage);
    if (!total_ms && !launches) return fail(P2O_ERR_ARG, "both outputs are NULL");
    if (!p->pending.empty()) {
        if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
        p2o_status s = drain_profile(p);
        if (s) return s;
    }
    auto it = p->by_nrhs.find({stage, nrhs});
    if (total_ms) *total_ms = it == p->by_nrhs.end() ? 0.0 : it->second.first;
    if (launches) *launches = it == p->by_nrhs.end() ? 0 : it->second.second;
    return P2O_OK;
}

p2o_status p2o_destroy(p2o_plan* plan) {
    if (!plan) return fail(P2O_ERR_ARG, "plan is NULL");
    delete plan;
    return P2O_OK;
}

p2o_status p2o_get_layout(const p2o_plan* p, int64_t* L, int64_t* nfreq, int64_t* pitch, int64_t* nscale_blocks) {
    if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
    if (L) *L = p->L;
    if (nfreq) *nfreq = p->nfreq;
    if (pitch) *pitch = p->pitch;
    if (nscale_blocks) *nscale_blocks = p->nblk;
    return P2O_OK;
}

p2o_status p2o_required_bytes(const p2o_plan* p, size_t* fhat_bytes, size_t* workspace_bytes) {
    if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
    if (!fhat_bytes && !workspace_bytes) return fail(P2O_ERR_ARG, "both outputs are NULL");
    if (fhat_bytes) *fhat_bytes = p->fhat_total;
    if (workspace_bytes) *workspace_bytes = p->ws_total;
    return P2O_OK;
}

p2o_status p2o_bind_storage(p2o_plan* p, void* fhat, size_t fhat_bytes, void* workspace, size_t workspace_bytes) {
    try {
        if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
        if (!fhat || !workspace) return fail(P2O_ERR_ARG, "storage pointer is NULL");
        if ((reinterpret_cast<uintptr_t>(fhat) | reinterpret_cast<uintptr_t>(workspace)) % kAlign)
            return fail(P2O_ERR_ARG, "storage must be %zu-byte aligned", kAlign);
        if (fhat_bytes < p->fhat_total || workspace_bytes < p->ws_total)
            return fail(P2O_ERR_STORAGE, "storage too small: spectrum %zu < %zu or workspace %zu < %zu", fhat_bytes,
                        p->fhat_total, workspace_bytes, p->ws_total);
        if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
        for (void* ptr : {fhat, workspace}) {
            hipPointerAttribute_t at;
            if (hipPointerGetAttributes(&at, ptr) != hipSuccess || at.type != hipMemoryTypeDevice) {
                (void)hipGetLastError();
                return fail(P2O_ERR_ARG, "storage pointer %p is not device memory", ptr);
            }
        }
        p->fhat = static_cast<char*>(fhat);
        p->ws = static_cast<char*>(workspace);
        p->state = kBound;
        p->aux_ready = false;
        std::fill(p->loaded.begin(), p->loaded.end(), 0);
        return P2O_OK;
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_bind_storage");
    }
}

p2o_status p2o_set_stream(p2o_plan* p, void* stream) {
    if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
    p->stream = static_cast<hipStream_t>(stream);
    return P2O_OK;
}

p2o_status p2o_load_blocks(p2o_plan* p, const void* F_chunk, int64_t col0, int64_t ncols, int32_t src_dtype) {
    try {
        if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
        if (!F_chunk) return fail(P2O_ERR_ARG, "F_chunk is NULL");
        if (src_dtype != P2O_SRC_F64 && src_dtype != P2O_SRC_F32)
            return fail(P2O_ERR_DTYPE, "unknown source dtype %d", (int)src_dtype);
        if (col0 < 0 || ncols < 1 || col0 + ncols > p->Nm)
            return fail(P2O_ERR_ARG, "columns [%lld, %lld) outside [0, Nm=%lld)", (long long)col0,
                        (long long)(col0 + ncols), (long long)p->Nm);
        if (ncols > (1LL << 30)) return fail(P2O_ERR_ARG, "ncols too large");
        const bool scaled = p->prec == P2O_BF16 || p->prec == P2O_FP16;
        if (scaled && (col0 % kScaleBlock != 0 || (ncols % kScaleBlock != 0 && col0 + ncols != p->Nm)))
            return fail(P2O_ERR_ARG, "BF16/FP16 loads need whole %d-column scale blocks (col0=%lld ncols=%lld)",
                        kScaleBlock, (long long)col0, (long long)ncols);
        if (p->state == kCreated) return fail(P2O_ERR_STATE, "bind storage before loading");
        if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
        p2o_status s;
        if (!p->aux_ready) {
            s = check_hip(launch_twiddle(p->fhat + p->off_tw64, p->fhat + p->off_tw32, (int)p->L, p->stream), "twiddles");
            if (s) return s;
            s = check_hip(hipMemsetAsync(p->fhat + p->off_flag, 0, sizeof(unsigned), p->stream), "flag reset");
            if (s) return s;
            s = check_hip(launch_zero_pad(p->fhat, p->nfreq * p->Nd, (int)p->pitch, (int)p->Nm, p->elem_bytes, p->stream),
                          "spectrum padding");
            if (s) return s;
            p->aux_ready = true;
        }
        LoadArgs la{};
        la.fhat = p->fhat;
        la.scales = reinterpret_cast<float*>(p->fhat + p->off_scales);
        la.flag = reinterpret_cast<unsigned*>(p->fhat + p->off_flag);
        la.col0 = col0;
        la.ncols = (int)ncols;
        la.Nd = (int)p->Nd;
        la.Nt = (int)p->Nt;
        la.t_stride = p->Nd * ncols;
        la.pitch = p->pitch;
        la.nblk = (int)p->nblk;
        la.rows_per_wg = (int)(p->Nd < 32 ? p->Nd : 32);
        s = staged(p, P2O_STAGE_LOAD, "spectrum load", [&] {
            return launch_load(p->prec, src_dtype == P2O_SRC_F64, p->fft, la, F_chunk, p->fhat + p->off_tw64, p->stream);
        });
        if (s) return s;
        std::fill(p->loaded.begin() + col0, p->loaded.begin() + col0 + ncols, 1);
        p->cur_nrhs = 0;
        p->state = kLoading;
        return P2O_OK;
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_load_blocks");
    }
}

p2o_status p2o_load_finalize(p2o_plan* p) {
    try {
        if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
        if (p->state != kLoading && p->state != kReady) return fail(P2O_ERR_STATE, "nothing loaded");
        for (size_t j = 0; j < p->loaded.size(); ++j)
            if (!p->loaded[j]) return fail(P2O_ERR_STATE, "column %zu of the blocks was never loaded", j);
        if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
        unsigned flag = 0;
        p2o_status s = check_hip(hipMemcpyAsync(&flag, p->fhat + p->off_flag, sizeof(flag), hipMemcpyDeviceToHost,
                                                p->stream), "flag readback");
        if (s) return s;
        s = check_hip(hipStreamSynchronize(p->stream), "load synchronisation");
        if (s) return s;
        if (flag) {
            p->state = kBound;
            p->aux_ready = false;
            std::fill(p->loaded.begin(), p->loaded.end(), 0);
            return fail(P2O_ERR_NONFINITE, "NaN or Inf in the time-domain blocks");
        }
        p->state = kReady;
        return P2O_OK;
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_load_finalize");
    }
}

p2o_status p2o_apply_F(p2o_plan* p, const void* m, void* d, int64_t nrhs, const int32_t* nt_active) {
    try {
        p2o_status s = ready_for_apply(p, m, d, nrhs);
        if (s) return s;
        if (p->qstride > 1) {
            if (nt_active) return fail(P2O_ERR_ARG, "ragged lengths are not defined with an output stride");
            s = enqueue_apply_F(p, m, p->ws + p->off_D2, nrhs, nullptr);
            return s ? s : qoi_sample(p, p->ws + p->off_D2, d, nrhs);
        }
        return enqueue_apply_F(p, m, d, nrhs, nt_active);
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_apply_F");
    }
}

p2o_status p2o_apply_F_noalloc(p2o_plan* p, const void* m, void* d, int64_t nrhs, const int32_t* nt_active) {
    try {
        p2o_status s = ready_for_apply(p, m, d, nrhs);
        if (s) return s;
        s = every_step(p, "p2o_apply_F_noalloc");
        if (s) return s;
        // the workspace layout for exactly nrhs right-hand sides, carved from
        // this device's scratch array for the duration of the call
        p2o_plan::Carve saved = p->carve;
        const int64_t saved_rhs = p->max_rhs;
        p->max_rhs = nrhs;
        layout(p);
        const size_t need = p->ws_total;
        char* const saved_ws = p->ws;
        auto restore = [&] {
            p->max_rhs = saved_rhs;
            p->carve = saved;
            p->ws = saved_ws;
        };
        if (need > kScratchBytes) {
            restore();
            return fail(P2O_ERR_ARG, "p2o_apply_F_noalloc: %lld right-hand sides need %zu bytes of scratch, more than "
                        "its %zu", (long long)nrhs, need, kScratchBytes);
        }
        void* scr = nullptr;
        s = scratch_on_current_device(p, &scr);
        if (s) {
            restore();
            return s;
        }
        p->ws = static_cast<char*>(scr);
        s = enqueue_apply_F(p, m, d, nrhs, nt_active);
        restore();
        return s;
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_apply_F_noalloc");
    }
}

p2o_status p2o_apply_Ft(p2o_plan* p, const void* d, void* m, int64_t nrhs, const int32_t* nt_active) {
    try {
        p2o_status s = ready_for_apply(p, d, m, nrhs);
        if (s) return s;
        if (p->qstride > 1) {
            if (nt_active) return fail(P2O_ERR_ARG, "ragged lengths are not defined with an output stride");
            s = qoi_expand(p, d, p->ws + p->off_D, nrhs);
            return s ? s : enqueue_apply_Ft(p, p->ws + p->off_D, m, nrhs, nullptr);
        }
        return enqueue_apply_Ft(p, d, m, nrhs, nt_active);
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_apply_Ft");
    }
}

p2o_status p2o_apply_FFt(p2o_plan* p, const void* e, void* h, int64_t nrhs, const int32_t* nt_active) {
    try {
        p2o_status s = ready_for_apply(p, e, h, nrhs);
        if (s) return s;
        if (p->qstride > 1) {
            if (nt_active) return fail(P2O_ERR_ARG, "ragged lengths are not defined with an output stride");
            s = qoi_expand(p, e, p->ws + p->off_D, nrhs);
            if (!s) s = enqueue_FFt(p, p->ws + p->off_D, p->ws + p->off_D2, nrhs, nullptr);
            return s ? s : qoi_sample(p, p->ws + p->off_D2, h, nrhs);
        }
        return enqueue_FFt(p, e, h, nrhs, nt_active);
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_apply_FFt");
    }
}

p2o_status p2o_assemble_K(p2o_plan* p, double prior_var, const double* noise_var, int64_t noise_var_len, double* K,
                          int64_t ldk, int64_t j0, int64_t ncols) {
    try {
        if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
        if (!K || !noise_var) return fail(P2O_ERR_ARG, "K or noise_var is NULL");
        int var_mode;
        p2o_status s = noise_mode(p, noise_var_len, &var_mode);
        if (s) return s;
        if (!(prior_var > 0.0) || prior_var > 1e300) return fail(P2O_ERR_ARG, "prior_var must be positive and finite");
        const int64_t N = p->Nt * p->Nd;
        if (ldk < N) return fail(P2O_ERR_ARG, "ldk=%lld < Nt*Nd=%lld", (long long)ldk, (long long)N);
        if (j0 < 0 || ncols < 1 || j0 + ncols > N)
            return fail(P2O_ERR_ARG, "columns [%lld, %lld) outside [0, %lld)", (long long)j0, (long long)(j0 + ncols),
                        (long long)N);
        s = ready_for_apply(p, K, K, ncols);
        if (!s) s = every_step(p, "p2o_assemble_K");
        if (s) return s;
        p->cur_nrhs = ncols;
        void* E = p->ws + p->off_D;
        void* H = p->ws + p->off_D2;
        const bool f64 = f64_plan(p);
        // gamma e_j: F (gamma F* e_j) is the column of F G* with G* = gamma F*
        s = check_hip(launch_unit_vectors(f64, E, N, j0, (int)ncols, prior_var, p->stream), "unit vectors");
        if (s) return s;
        s = enqueue_FFt(p, E, H, ncols, nullptr);
        if (s) return s;
        return check_hip(launch_K_columns(f64, H, N, K, ldk, j0, (int)ncols, noise_var, var_mode, (int)p->Nd, p->stream),
                         "K columns");
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_assemble_K");
    }
}

p2o_status p2o_gram_accumulate(const double* blocks, int64_t Nt, int64_t Nd, int64_t ncols, int64_t ldb, double* G,
                               int64_t ldg, void* stream) {
    if (!blocks || !G) return fail(P2O_ERR_ARG, "blocks or G is NULL");
    if (Nt < 1 || Nd < 1 || Nt * Nd > (1LL << 31) - 1) return fail(P2O_ERR_ARG, "Nt=%lld, Nd=%lld invalid", (long long)Nt, (long long)Nd);
    const int64_t N = Nt * Nd;
    if (ncols < 1 || ncols > (1LL << 31) - 1 || ldb < ncols || ldg < N)
        return fail(P2O_ERR_ARG, "ncols=%lld, ldb=%lld or ldg=%lld invalid", (long long)ncols, (long long)ldb,
                    (long long)ldg);
    if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
    return check_hip(launch_gram_update(blocks, ldb, N, (int)ncols, G, ldg, static_cast<hipStream_t>(stream)),
                     "Gram update");
}

p2o_status p2o_gram_to_K(double* G, int64_t ldg, int64_t Nt, int64_t Nd, double prior_var, const double* noise_var,
                         int64_t noise_var_len, void* stream) {
    if (!G || !noise_var) return fail(P2O_ERR_ARG, "G or noise_var is NULL");
    if (Nt < 1 || Nd < 1 || Nt * Nd > (1LL << 31) - 1) return fail(P2O_ERR_ARG, "Nt=%lld, Nd=%lld invalid", (long long)Nt, (long long)Nd);
    if (ldg < Nt * Nd) return fail(P2O_ERR_ARG, "ldg=%lld < Nt*Nd=%lld", (long long)ldg, (long long)(Nt * Nd));
    if (!(prior_var > 0.0) || prior_var > 1e300) return fail(P2O_ERR_ARG, "prior_var must be positive and finite");
    int var_mode;
    if (noise_var_len == 1) var_mode = 0;
    else if (noise_var_len == Nd) var_mode = 1;
    else if (noise_var_len == Nd * Nt) var_mode = 2;
    else
        return fail(P2O_ERR_ARG, "noise_var_len=%lld must be 1, Nd=%lld or Nt*Nd=%lld", (long long)noise_var_len,
                    (long long)Nd, (long long)(Nd * Nt));
    if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
    return check_hip(launch_gram_to_K(G, ldg, (int)Nt, (int)Nd, prior_var, noise_var, var_mode,
                                      static_cast<hipStream_t>(stream)),
                     "K from the Gram matrix");
}

p2o_status p2o_cholesky(double* A, int64_t n, int64_t lda, int32_t* info, void* stream) {
    if (!A || !info) return fail(P2O_ERR_ARG, "A or info is NULL");
    if (n < 1 || n > (1LL << 31) - 1 || lda < n) return fail(P2O_ERR_ARG, "n=%lld or lda=%lld invalid", (long long)n, (long long)lda);
    if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
    return check_hip(launch_cholesky(A, n, lda, info, static_cast<hipStream_t>(stream)), "Cholesky factorisation");
}

p2o_status p2o_cholesky_solve(const double* L, int64_t n, int64_t lda, double* X, int64_t nrhs, int64_t ldx,
                              void* stream) {
    if (!L || !X) return fail(P2O_ERR_ARG, "L or X is NULL");
    if (n < 1 || n > (1LL << 31) - 1 || lda < n || ldx < n)
        return fail(P2O_ERR_ARG, "n=%lld, lda=%lld or ldx=%lld invalid", (long long)n, (long long)lda, (long long)ldx);
    if (nrhs < 1 || nrhs > 65535) return fail(P2O_ERR_ARG, "nrhs=%lld outside [1, 65535]", (long long)nrhs);
    if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
    return check_hip(launch_cholesky_solve(L, n, lda, X, (int)nrhs, ldx, static_cast<hipStream_t>(stream)),
                     "Cholesky solve");
}

p2o_status p2o_map_point(p2o_plan* p, double prior_var, const double* noise_var, int64_t noise_var_len,
                         const double* L, int64_t ldl, const void* d_obs, void* m_map, int64_t nrhs) {
    try {
        if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
        if (!L || !noise_var) return fail(P2O_ERR_ARG, "L or noise_var is NULL");
        int var_mode;
        p2o_status s = noise_mode(p, noise_var_len, &var_mode);
        if (s) return s;
        if (!(prior_var > 0.0) || prior_var > 1e300) return fail(P2O_ERR_ARG, "prior_var must be positive and finite");
        const int64_t N = p->Nt * p->Nd;
        if (ldl < N) return fail(P2O_ERR_ARG, "ldl=%lld < Nt*Nd=%lld", (long long)ldl, (long long)N);
        s = ready_for_apply(p, d_obs, m_map, nrhs);
        if (!s) s = every_step(p, "p2o_map_point");
        if (s) return s;
        p->cur_nrhs = nrhs;
        const bool f64 = f64_plan(p);
        void* D = p->ws + p->off_D;
        void* D2 = p->ws + p->off_D2;
        double* Z = reinterpret_cast<double*>(p->ws + p->off_Z);
        // w = gamma Gamma_noise^{-1} d; u = F* w (= G* Gamma_noise^{-1} d)
        s = check_hip(launch_weight_data(f64, d_obs, D, N, (int)nrhs, noise_var, var_mode, (int)p->Nd, prior_var,
                                         p->stream), "noise weighting");
        if (!s) s = enqueue_apply_Ft(p, D, m_map, nrhs, nullptr);
        // z = K^{-1} F u
        if (!s) s = enqueue_apply_F(p, m_map, D2, nrhs, nullptr);
        if (!s) s = check_hip(launch_to_f64(f64, D2, Z, N, (int)nrhs, N, p->stream), "data vectors to FP64");
        if (!s) s = check_hip(launch_cholesky_solve(L, N, ldl, Z, (int)nrhs, N, p->stream), "K solve");
        // m_map = G* (Gamma_noise^{-1} d - z) = F* (w - gamma z)
        if (!s) s = check_hip(launch_combine(f64, D, Z, N, (int)nrhs, N, 1.0, -prior_var, p->stream), "w - gamma z");
        if (!s) s = enqueue_apply_Ft(p, D, m_map, nrhs, nullptr);
        return s;
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_map_point");
    }
}

p2o_status p2o_posterior_cov_apply(p2o_plan* p, double prior_var, const double* L, int64_t ldl, const void* v,
                                   void* out, int64_t nrhs) {
    try {
        if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
        if (!L) return fail(P2O_ERR_ARG, "L is NULL");
        if (!(prior_var > 0.0) || prior_var > 1e300) return fail(P2O_ERR_ARG, "prior_var must be positive and finite");
        const int64_t N = p->Nt * p->Nd;
        if (ldl < N) return fail(P2O_ERR_ARG, "ldl=%lld < Nt*Nd=%lld", (long long)ldl, (long long)N);
        p2o_status s = ready_for_apply(p, v, out, nrhs);
        if (!s) s = every_step(p, "p2o_posterior_cov_apply");
        if (s) return s;
        if (v == out) return fail(P2O_ERR_ARG, "v and out must not be the same buffer");
        p->cur_nrhs = nrhs;
        const bool f64 = f64_plan(p);
        const long long nm = (long long)nrhs * p->Nt * p->Nm;
        void* D = p->ws + p->off_D;
        void* D2 = p->ws + p->off_D2;
        double* Z = reinterpret_cast<double*>(p->ws + p->off_Z);
        // w = gamma v (Gamma_prior v); z = K^{-1} F w
        s = check_hip(launch_axpby(f64, v, out, nm, 0.0, prior_var, p->stream), "gamma v");
        if (!s) s = enqueue_apply_F(p, out, D2, nrhs, nullptr);
        if (!s) s = check_hip(launch_to_f64(f64, D2, Z, N, (int)nrhs, N, p->stream), "data vectors to FP64");
        if (!s) s = check_hip(launch_cholesky_solve(L, N, ldl, Z, (int)nrhs, N, p->stream), "K solve");
        // out = w - G* z = F* (-gamma z) + gamma v
        if (!s) s = check_hip(launch_combine(f64, D, Z, N, (int)nrhs, N, 0.0, -prior_var, p->stream), "-gamma z");
        if (!s) s = enqueue_apply_Ft(p, D, out, nrhs, nullptr);
        if (!s) s = check_hip(launch_axpby(f64, v, out, nm, 1.0, prior_var, p->stream), "+ gamma v");
        return s;
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_posterior_cov_apply");
    }
}

p2o_status p2o_apply_FGt(p2o_plan* F, p2o_plan* G, const void* e, void* h, int64_t nrhs) {
    try {
        p2o_status s = compatible(F, G, nrhs);
        if (s) return s;
        if (!e || !h) return fail(P2O_ERR_ARG, "input or output pointer is NULL");
        const void* e_full = e;
        if (G->qstride > 1) {
            s = qoi_expand(G, e, G->ws + G->off_D, nrhs);
            if (s) return s;
            e_full = G->ws + G->off_D;
        }
        void* h_full = F->qstride > 1 ? F->ws + F->off_D2 : h;
        s = enqueue_cross(F, G, e_full, h_full, nrhs);
        if (s) return s;
        return F->qstride > 1 ? qoi_sample(F, h_full, h, nrhs) : P2O_OK;
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_apply_FGt");
    }
}

p2o_status p2o_d2q_rows(p2o_plan* F, p2o_plan* Fq, double prior_var, const double* noise_var, int64_t noise_var_len,
                        const double* L, int64_t ldl, int64_t r0, int64_t nrows, double* Q, int64_t ldq) {
    try {
        p2o_status s = compatible(F, Fq, nrows);
        if (s) return s;
        if (!L || !noise_var || !Q) return fail(P2O_ERR_ARG, "L, noise_var or Q is NULL");
        int var_mode;
        s = noise_mode(F, noise_var_len, &var_mode);
        if (!s) s = every_step(F, "the data side of p2o_d2q_rows");
        if (s) return s;
        if (!(prior_var > 0.0) || prior_var > 1e300) return fail(P2O_ERR_ARG, "prior_var must be positive and finite");
        const int64_t N = F->Nt * F->Nd, nq = (F->Nt / Fq->qstride) * Fq->Nd;
        if (ldl < N || ldq < N) return fail(P2O_ERR_ARG, "ldl=%lld or ldq=%lld < Nt*Nd=%lld", (long long)ldl, (long long)ldq, (long long)N);
        if (r0 < 0 || r0 + nrows > nq)
            return fail(P2O_ERR_ARG, "rows [%lld, %lld) outside [0, %lld)", (long long)r0, (long long)(r0 + nrows), (long long)nq);
        const bool f64 = f64_plan(F);
        // unit QoI vectors -> y = F F_q^* e_r (Fq's series expanded in its own workspace)
        void* E = Fq->ws + Fq->off_D2;
        s = check_hip(launch_unit_vectors(f64, E, nq, r0, (int)nrows, 1.0, F->stream), "unit vectors");
        const void* E_full = E;
        if (!s && Fq->qstride > 1) {
            s = qoi_expand(Fq, E, Fq->ws + Fq->off_D, nrows);
            E_full = Fq->ws + Fq->off_D;
        }
        void* Y = F->ws + F->off_D;
        void* H = F->ws + F->off_D2;
        double* Z = reinterpret_cast<double*>(F->ws + F->off_Z);
        if (!s) s = enqueue_cross(F, Fq, E_full, Y, nrows);
        // z = gamma K^{-1} y; h = F F^* z (= F G^* K^{-1} y)
        if (!s) s = check_hip(launch_to_f64(f64, Y, Z, N, (int)nrows, N, F->stream), "data vectors to FP64");
        if (!s) s = check_hip(launch_cholesky_solve(L, N, ldl, Z, (int)nrows, N, F->stream), "K solve");
        if (!s) s = check_hip(launch_combine(f64, H, Z, N, (int)nrows, N, 0.0, prior_var, F->stream), "gamma z");
        if (!s) s = enqueue_FFt(F, H, H, nrows, nullptr);
        // row = gamma Gamma_noise^{-1} (y - h)
        if (!s) s = check_hip(launch_d2q_rows(f64, Y, H, N, (int)nrows, Q, ldq, r0, noise_var, var_mode, (int)F->Nd,
                                              prior_var, F->stream), "d2q rows");
        return s;
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_d2q_rows");
    }
}

p2o_status p2o_qoi_posterior_cov(p2o_plan* F, p2o_plan* Fq, double prior_var, const double* L, int64_t ldl,
                                 int64_t c0, int64_t ncols, double* C, int64_t ldc) {
    try {
        p2o_status s = compatible(F, Fq, ncols);
        if (s) return s;
        if (!L || !C) return fail(P2O_ERR_ARG, "L or C is NULL");
        s = every_step(F, "the data side of p2o_qoi_posterior_cov");
        if (s) return s;
        if (!(prior_var > 0.0) || prior_var > 1e300) return fail(P2O_ERR_ARG, "prior_var must be positive and finite");
        const int64_t N = F->Nt * F->Nd, nq = (F->Nt / Fq->qstride) * Fq->Nd;
        if (ldl < N) return fail(P2O_ERR_ARG, "ldl=%lld < Nt*Nd=%lld", (long long)ldl, (long long)N);
        if (ldc < nq) return fail(P2O_ERR_ARG, "ldc=%lld < Nq*Ntq=%lld", (long long)ldc, (long long)nq);
        if (c0 < 0 || c0 + ncols > nq)
            return fail(P2O_ERR_ARG, "columns [%lld, %lld) outside [0, %lld)", (long long)c0, (long long)(c0 + ncols),
                        (long long)nq);
        const bool f64 = f64_plan(F);
        const int rq = Fq->qstride;
        void* E = Fq->ws + Fq->off_D2;
        void* Efull = Fq->ws + Fq->off_D;
        s = check_hip(launch_unit_vectors(f64, E, nq, c0, (int)ncols, 1.0, F->stream), "unit vectors");
        if (!s) s = qoi_expand(Fq, E, Efull, ncols);           // stride 1: a copy
        // y = F F_q^* e_c
        void* Y = F->ws + F->off_D;
        double* Z = reinterpret_cast<double*>(F->ws + F->off_Z);
        if (!s) s = enqueue_cross(F, Fq, Efull, Y, ncols);
        // C[:, c] = gamma F_q F_q^* e_c ...
        if (!s) s = enqueue_FFt(Fq, Efull, Efull, ncols, nullptr);
        if (!s) s = check_hip(launch_qoi_gather(f64, Efull, nullptr, C, ldc, c0, prior_var, false, (int)Fq->Nt,
                                                (int)Fq->Nd, rq, (int)ncols, F->stream), "QoI columns");
        // ... - gamma F_q G^* K^{-1} y, G^* = gamma F^*
        if (!s) s = check_hip(launch_to_f64(f64, Y, Z, N, (int)ncols, N, F->stream), "data vectors to FP64");
        if (!s) s = check_hip(launch_cholesky_solve(L, N, ldl, Z, (int)ncols, N, F->stream), "K solve");
        void* W = F->ws + F->off_D2;
        if (!s) s = check_hip(launch_combine(f64, W, Z, N, (int)ncols, N, 0.0, prior_var, F->stream), "gamma z");
        if (!s) s = enqueue_cross(Fq, F, W, Efull, ncols);
        if (!s) s = check_hip(launch_qoi_gather(f64, Efull, nullptr, C, ldc, c0, -prior_var, true, (int)Fq->Nt,
                                                (int)Fq->Nd, rq, (int)ncols, F->stream), "QoI columns");
        return s;
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_qoi_posterior_cov");
    }
}

p2o_status p2o_d2q_apply(const double* Q, int64_t nq, int64_t N, int64_t ldq, const double* d, double* q, int64_t nrhs,
                         void* stream) {
    if (!Q || !d || !q) return fail(P2O_ERR_ARG, "Q, d or q is NULL");
    if (nq < 1 || N < 1 || ldq < N || nrhs < 1 || nrhs > 65535)
        return fail(P2O_ERR_ARG, "nq=%lld, N=%lld, ldq=%lld or nrhs=%lld invalid", (long long)nq, (long long)N,
                    (long long)ldq, (long long)nrhs);
    if (!have_device()) return fail(P2O_ERR_NO_DEVICE, "no GPU available");
    return check_hip(launch_d2q_apply(Q, nq, N, ldq, d, q, (int)nrhs, static_cast<hipStream_t>(stream)), "Q d");
}

p2o_status p2o_misfit_grad(p2o_plan* p, const void* m, const void* d_obs, const double* noise_var,
                           int64_t noise_var_len, void* grad, double* misfit, int64_t nrhs, const int32_t* nt_active) {
    try {
        if (!p) return fail(P2O_ERR_ARG, "plan is NULL");
        if (!d_obs || !noise_var || !misfit) return fail(P2O_ERR_ARG, "d_obs, noise_var or misfit is NULL");
        int var_mode;
        p2o_status s = noise_mode(p, noise_var_len, &var_mode);
        if (s) return s;
        s = ready_for_apply(p, m, grad, nrhs);
        if (!s) s = every_step(p, "p2o_misfit_grad");
        if (s) return s;
        p->cur_nrhs = nrhs;
        s = enqueue_forward_to_Y(p, m, nrhs, nt_active);
        if (s) return s;
        void* D = p->ws + p->off_D;
        double* P = reinterpret_cast<double*>(p->ws + p->off_P);
        s = staged(p, P2O_STAGE_C2R, "c2r with misfit", [&] {
            return launch_c2r(f64_plan(p), p->fft, io_data(p, nrhs, nt_active, fwd_parts(p, nrhs)), p->ws + p->off_Y, D,
                              tw_of(p), d_obs, noise_var, var_mode, P, p->stream);
        });
        if (s) return s;
        s = staged(p, P2O_STAGE_REDUCE, "misfit reduction", [&] {
            return launch_misfit_reduce(P, p->c2r_nd_blocks, misfit, (int)nrhs, p->stream);
        });
        if (s) return s;
        s = enqueue_adjoint_to_X(p, D, nrhs, nt_active);
        if (s) return s;
        return staged(p, P2O_STAGE_C2R, "c2r (gradient)", [&] {
            return launch_c2r(f64_plan(p), p->fft, io_param(p, nrhs, nt_active, adj_parts(p, nrhs)), p->ws + p->off_X, grad,
                              tw_of(p), nullptr, nullptr, 0, nullptr, p->stream);
        });
    } catch (...) {
        return fail(P2O_ERR_ARG, "internal error in p2o_misfit_grad");
    }
}

}  // extern "C"
