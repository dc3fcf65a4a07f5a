// Batched per-frequency products on the matrix cores (many right-hand sides
// per launch): Y_w = Fhat_w X_w and X'_w = Fhat_w^H Y_w for a BF16 spectrum.
//
// With B right-hand sides the per-frequency matvecs of section 4 become one
// complex GEMM per frequency, done with v_mfma_f32_32x32x16_bf16 (on gfx950
// the 32x32 shape sustains about 1.5x the rate of the 16x16x32 one, and
// does so with one wavefront per SIMD).  K runs over (index, re/im) pairs in
// their stored interleaved order, so a complex product is two real ones of
// the stored spectrum fragment against forms of the right-hand-side
// fragment, each 32-bit word (re, im) being rewritten by one or two VALU
// operations (a right-hand-side fragment serves MB spectrum fragments, so
// the forms cost a fraction of what forms of the spectrum would):
//   forward  y_r = (a_r, a_i) . (x_r, -x_i)   y_i = (a_r, a_i) . (x_i, x_r)
//   adjoint  x_r = (a_r, a_i) . (y_r,  y_i)   x_i = (a_r, a_i) . (y_i, -y_r)
// (the adjoint takes conj(F)^T).  With a BF16 spectrum the right-hand sides
// arrive as quad BF16 hi/lo storage (written by the FFT that produced them);
// hi and lo each go through the matrix cores, giving about 16 significant
// bits of x with FP32 accumulation.  With an FP16 spectrum (LDS-ring kernels
// only) they arrive as complex FP32, and each fragment is rounded to FP16
// after multiplying by its right-hand side's power-of-two scale (which maps
// that right-hand side's largest entry into (2^14, 2^15]), one
// v_mfma_f32_32x32x16_f16 per form: half the matrix-core work of the BF16
// hi + lo products, at FP16's 11 significant bits on both operands.  The
// per-(frequency, 4096-column block) power-of-two scale of the stored
// spectrum, and the inverse right-hand-side scale, multiply finished outputs
// (exact).
//
// Work.  A workgroup is NW (4 or 8) wavefronts: RG row groups x (NW / RG)
// halves of the right-hand sides, each wavefront computing MB (4 or 5) blocks
// of 32 output rows (forward: sensors; adjoint: parameter columns) for 32
// right-hand sides.
// Each K step (KU substeps of 8 complex entries) the workgroup stages its
// spectrum tile and right-hand-side tile in LDS, loaded cooperatively with
// whole 128-byte lines per 8 lanes: forward rows in runs of 32 (or 16)
// columns, adjoint sensor rows of 256 to 640 contiguous columns.  In the
// register-staged kernel (k_gemm) loads run two steps ahead through
// registers into a double buffer; the LDS-ring kernels (k_gemm_fwd_ring,
// k_gemm_adj_ring, the built-in choice) load straight into a 3-step ring in
// LDS.  One barrier per step separates staging from the matrix-core work.
// Fragments
// come from padded LDS rows without bank conflicts: forward lanes read 16
// bytes of a row, adjoint lanes gather 4 sensors of a column as 4-byte words.
// Every spectrum byte is read once per launch.  Forward workgroups own
// (frequency, 4096-column chunk, row tile, right-hand-side group) and write
// the chunk's partial products to their own slot (summed in fixed order by
// the inverse FFT); adjoint workgroups own (frequency, column tile,
// right-hand-side group).  Workgroup ids are mapped so that consecutive ids
// on one XCD share the frequency (and forward column chunk): the
// right-hand-side spectra they all read stay in that XCD's L2.
#include "common.hpp"
#include "kernels.hpp"

namespace p2o {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));   // native vector: staged copies stay in registers


__device__ __forceinline__ f32x16 mfma32(uint4 a, uint4 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                   c, 0, 0, 0);
}

// forms of a fragment of (re, im) BF16 words
__device__ __forceinline__ uint32_t w_swap(uint32_t w) { return __builtin_amdgcn_alignbit(w, w, 16); }
__device__ __forceinline__ uint4 f_conj(uint4 a) {                       // (re, -im)
    return make_uint4(a.x ^ 0x80000000u, a.y ^ 0x80000000u, a.z ^ 0x80000000u, a.w ^ 0x80000000u);
}
__device__ __forceinline__ uint4 f_swap(uint4 a) {                       // (im, re)
    return make_uint4(w_swap(a.x), w_swap(a.y), w_swap(a.z), w_swap(a.w));
}
__device__ __forceinline__ uint4 f_nswap(uint4 a) {                      // (im, -re)
    return make_uint4(w_swap(a.x) ^ 0x80000000u, w_swap(a.y) ^ 0x80000000u, w_swap(a.z) ^ 0x80000000u,
                      w_swap(a.w) ^ 0x80000000u);
}

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x16 mfma32h(uint4 a, uint4 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0,
                                                  0);
}

// (re, im) FP32 -> one word of two FP16 (nearest even, one v_cvt_pk_f16_f32),
// after multiplying by the right-hand side's scale s (a power of two: exact).
__device__ __forceinline__ uint32_t w_f16(uint32_t re, uint32_t im, float s) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{__uint_as_float(re) * s,
                                                                        __uint_as_float(im) * s}, f16x2));
}
// (re, im) FP32 times s as one word of two FP16 (nearest even).
__device__ __forceinline__ uint32_t pack_f16(float re, float im, float s) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{re * s, im * s}, f16x2));
}
// Four consecutive complex FP32 values (two 16-byte parts) as an FP16 fragment.
__device__ __forceinline__ uint4 f_rhs_f16(uint4 p0, uint4 p1, float s) {
    return make_uint4(w_f16(p0.x, p0.y, s), w_f16(p0.z, p0.w, s), w_f16(p1.x, p1.y, s), w_f16(p1.z, p1.w, s));
}

__device__ __forceinline__ int xcd_item(int id, int Q) { return (id & 7) * Q + (id >> 3); }

// Workgroup barrier that waits for this wavefront's LDS operations but not
// for its loads in flight (__syncthreads would also drain the prefetch).  The
// empty asm statements keep the compiler from moving memory accesses across.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);      // lgkmcnt(0); vmcnt, expcnt not waited on
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Tile geometry.  FWD: the A tile is MROWS rows x KC columns, row stride
// A_RS bytes (16 bytes of padding: the 16-byte fragment reads of 16
// consecutive rows hit distinct banks).  ADJ: KC sensor rows x MROWS columns,
// row stride A_RS with 4 A_RS / 4 = 32 (mod 64) banks, so the two sensor
// quartets a fragment read covers fall in different bank halves.
template <bool FWD, int RG, int KU, int MB_, int NW>
struct Tile {
    static constexpr int THREADS = 64 * NW;            // NW wavefronts = RG row groups x NH halves
    static constexpr int MB = MB_;                     // 32-row blocks per wavefront
    static constexpr int NH = NW / RG;                 // right-hand-side halves of 32
    static constexpr int MROWS = RG * 32 * MB;         // output rows per workgroup
    static constexpr int KC = 8 * KU;                  // complex K entries per step
    static constexpr int RHS = 32 * NH;
    static constexpr int A_RS = FWD ? KC * 4 + 16 : MROWS * 4 + 32;
    static constexpr int A_BYTES = FWD ? MROWS * A_RS : KC * A_RS;
    static constexpr int A_CPR = FWD ? KC / 4 : MROWS / 4;   // 16-byte chunks per stored row
    static constexpr int A_PT = MROWS * KC / 4 / THREADS;
    static constexpr int B_PT = RHS * KC / 2 / THREADS;    // 16-byte hi or lo chunks
    static_assert(A_PT * THREADS * 4 == MROWS * KC, "A chunks per thread");
    static_assert(B_PT * THREADS * 2 == RHS * KC, "B chunks per thread");
};

// LDS slot of lane L's B fragment in plane (substep u, hi/lo hl): the low 4
// bits are rotated by 4 u + 2 hl + L / 32, so that the 16 chunks one
// right-hand side contributes per step (8 groups x hi/lo) land in 16
// different bank groups when stored, while the 64 lanes of a fragment read
// still cover one contiguous kilobyte.
__device__ __forceinline__ int b_slot(int L, int u, int hl) { return (L & 48) | ((L + 4 * u + 2 * hl + (L >> 5)) & 15); }

// Registers of one staged step (A and B chunks, B validity masks).
template <int AP, int BP>
struct Staged {
    v4u a[AP];
    v4u b[BP];
    uint32_t m[BP];
};

// WPE: wavefronts per SIMD the register allocation must allow (2: the
// accumulators share the 256 registers of a wavefront with everything else).
// PF: steps staged in registers ahead of the LDS double buffer (2, or 1 to
// fit two wavefronts per SIMD; the other workgroup on the CU then covers the
// shorter lead).
template <bool FWD, int RG, int KU, int MB_, int WPE, int PF, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE)))
void k_gemm(const uint8_t* fhat, const float* __restrict__ scales, const uint8_t* Bq, float2* __restrict__ out_base,
            GemmArgs ga) {
    using T = Tile<FWD, RG, KU, MB_, NW>;
    constexpr int MB = MB_;
    __shared__ __align__(16) uint8_t as[2][T::A_BYTES];
    __shared__ __align__(16) v4u bfr[2][KU][T::NH][2][64];

    const int q = xcd_item(blockIdx.x, ga.Q);
    if (q >= ga.items) return;
    int t = q;
    const int mt = t % ga.n_mt; t /= ga.n_mt;
    const int bg = t % ga.n_bg; t /= ga.n_bg;
    const int kc = t % ga.n_kc; t /= ga.n_kc;
    const int w = t;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rg = wave % RG, nh = wave / RG;
    const int r = lane & 31, kg = lane >> 5;
    const int b0 = bg * T::RHS;
    const int nb_valid = min(T::RHS, ga.nrhs - b0);
    const int m0 = mt * T::MROWS;                      // first output row (sensor or column) of the tile
    // K range: forward columns [kbeg, kend) of the chunk, adjoint sensors [0, ldb)
    const int kbeg = FWD ? kc * ga.kchunk : 0;
    const int kend = FWD ? min(ga.ncols, kbeg + ga.kchunk) : ga.ldb;
    const int nst = (kend - kbeg + T::KC - 1) / T::KC;
    const uint32_t* Fw = reinterpret_cast<const uint32_t*>(fhat) + (long long)w * ga.Nd * ga.pitch;
    const uint8_t* brows = Bq + ((long long)w * ga.nrhs + b0) * ga.ldb * 8;
    const long long ldb_bytes = (long long)ga.ldb * 8;

    using S = Staged<T::A_PT, T::B_PT>;
    // Loads of step st.  A: chunk c covers 4 consecutive entries of a stored
    // row (forward: sensor row m0 + c / A_CPR, columns from 4 (c % A_CPR);
    // adjoint: sensor row c / A_CPR, columns m0 + 4 (c % A_CPR)); rows past
    // Nd and columns past the chunk or the pitch read a valid address (their
    // B entries are zero or their outputs are not stored).  B: chunk c is the
    // hi (even c) or lo half of the 4-entry group g of right-hand side bl.
    auto load = [&](S& sg, int st) {
        const int sa = min(st, nst - 1);
#pragma unroll
        for (int i = 0; i < T::A_PT; ++i) {
            const int c = tid + i * T::THREADS;
            const int row = c / T::A_CPR, cc = c % T::A_CPR;
            long long off;
            if constexpr (FWD) {
                const int sr = min(m0 + row, ga.Nd - 1);
                int j = kbeg + sa * T::KC + 4 * cc;
                if (j >= kend) j = kbeg;
                off = (long long)sr * ga.pitch + j;
            } else {
                const int sr = min(sa * T::KC + row, ga.Nd - 1);
                const int j = min(m0 + 4 * cc, ga.pitch - 4);
                off = (long long)sr * ga.pitch + j;
            }
            sg.a[i] = *reinterpret_cast<const v4u*>(Fw + off);
        }
#pragma unroll
        for (int i = 0; i < T::B_PT; ++i) {
            const int c = tid + i * T::THREADS;
            const int p = c >> 1, hl = c & 1;
            const int g = p % (T::KC / 4), bl = min(p / (T::KC / 4), nb_valid - 1);
            const int gi = (kbeg + st * T::KC) / 4 + g;
            const bool ok = gi < kend / 4;
            sg.b[i] = *reinterpret_cast<const v4u*>(brows + bl * ldb_bytes + (long long)(ok ? gi : 0) * 32 + hl * 16);
            sg.m[i] = ok ? 0xffffffffu : 0u;
        }
    };
    auto store = [&](const S& sg, int buf) {
#pragma unroll
        for (int i = 0; i < T::A_PT; ++i) {
            const int c = tid + i * T::THREADS;
            const int row = c / T::A_CPR, cc = c % T::A_CPR;
            *reinterpret_cast<v4u*>(&as[buf][row * T::A_RS + cc * 16]) = sg.a[i];
        }
#pragma unroll
        for (int i = 0; i < T::B_PT; ++i) {
            const int c = tid + i * T::THREADS;
            const int p = c >> 1, hl = c & 1;
            const int g = p % (T::KC / 4), bl = p / (T::KC / 4);
            // The empty asm pins the first use of the loaded chunk here: left
            // free, the compiler hoists the masking into the previous step,
            // whose wait for this load then drains the other step in flight.
            v4u v = sg.b[i];
            asm volatile("" : "+v"(v));
            bfr[buf][g >> 1][bl >> 5][hl][b_slot((bl & 31) + 32 * (g & 1), g >> 1, hl)] = v & sg.m[i];
        }
    };

    f32x16 accr[MB], acci[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) accr[mb] = acci[mb] = f32x16{};

    // A fragment of block mb, substep u: forward lane (r, kg) holds row r,
    // entries 4 kg .. 4 kg + 3 of the substep; adjoint lane (r, kg) holds
    // sensors 4 kg .. 4 kg + 3 of the substep for column r.
    auto frag = [&](int buf, int mb, int u) -> uint4 {
        const int mrow = (rg * MB + mb) * 32 + r;
        if constexpr (FWD) {
            const v4u v = *reinterpret_cast<const v4u*>(&as[buf][mrow * T::A_RS + (2 * u + kg) * 16]);
            return make_uint4(v.x, v.y, v.z, v.w);
        } else {
            const uint8_t* p = &as[buf][(8 * u + 4 * kg) * T::A_RS + mrow * 4];
            return make_uint4(*reinterpret_cast<const uint32_t*>(p),
                              *reinterpret_cast<const uint32_t*>(p + T::A_RS),
                              *reinterpret_cast<const uint32_t*>(p + 2 * T::A_RS),
                              *reinterpret_cast<const uint32_t*>(p + 3 * T::A_RS));
        }
    };
    auto compute = [&](int buf) {
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const v4u vh = bfr[buf][u][nh][0][b_slot(lane, u, 0)], vl = bfr[buf][u][nh][1][b_slot(lane, u, 1)];
            const uint4 bh = make_uint4(vh.x, vh.y, vh.z, vh.w), bl = make_uint4(vl.x, vl.y, vl.z, vl.w);
            const uint4 bh_r = FWD ? f_conj(bh) : bh, bl_r = FWD ? f_conj(bl) : bl;
            const uint4 bh_i = FWD ? f_swap(bh) : f_nswap(bh), bl_i = FWD ? f_swap(bl) : f_nswap(bl);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const uint4 a = frag(buf, mb, u);
                accr[mb] = mfma32(a, bh_r, accr[mb]);
                acci[mb] = mfma32(a, bh_i, acci[mb]);
                accr[mb] = mfma32(a, bl_r, accr[mb]);
                acci[mb] = mfma32(a, bl_i, acci[mb]);
            }
        }
    };

    // Step st: store step st+1 (loaded PF steps earlier) into the LDS buffer
    // step st-1 read; load step st+1+PF into the freed registers; compute
    // step st; barrier.  Loads retire in order and step st+1 was issued
    // before the later ones, so waiting for it leaves PF-1 steps in flight.
    // Loads past the last step repeat it (A) or read zeros (B) and are never
    // used.
    auto step = [&](S& sn, int buf, int st) {
        store(sn, buf ^ 1);
        load(sn, st + 1 + PF);
        compute(buf);
        lds_barrier();
    };
    if constexpr (PF == 2) {
        S s0, s1;
        load(s0, 0);
        load(s1, 1);
        store(s0, 0);
        load(s0, 2);
        lds_barrier();
        int st = 0;
        for (; st + 2 <= nst; st += 2) {
            step(s1, 0, st);
            step(s0, 1, st + 1);
        }
        if (st < nst) step(s1, 0, st);
    } else {
        S s0;
        load(s0, 0);
        store(s0, 0);
        load(s0, 1);
        lds_barrier();
        int st = 0;
        for (; st + 2 <= nst; st += 2) {
            step(s0, 0, st);
            step(s0, 1, st + 1);
        }
        if (st < nst) step(s0, 0, st);
    }

    // output tile (32 rows x 32 right-hand sides): lane (n, h) holds rows
    // 8 (v / 4) + 4 h + v % 4 of column n in element v
    const int b = b0 + 32 * nh + r;
    if (b >= ga.nrhs) return;
    if constexpr (FWD) {
        const float sc = scales[(long long)w * ga.nblk + kbeg / kScaleBlock];
        float2* out = out_base + (long long)kc * ga.part_stride + ((long long)w * ga.nrhs + b) * ga.Nd;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = m0 + (rg * MB + mb) * 32 + 8 * (v >> 2) + 4 * kg + (v & 3);
                if (row < ga.Nd) out[row] = make_float2(accr[mb][v] * sc, acci[mb][v] * sc);
            }
    } else {
        float2* out = out_base + ((long long)w * ga.nrhs + b) * ga.pitch;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int jb = m0 + (rg * MB + mb) * 32;        // an m block lies in one 4096-column scale block
            if (jb >= ga.ncols) continue;
            const float sc = scales[(long long)w * ga.nblk + jb / kScaleBlock];
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int j = jb + 8 * (v >> 2) + 4 * kg + (v & 3);
                if (j < ga.ncols) out[j] = make_float2(accr[mb][v] * sc, acci[mb][v] * sc);
            }
        }
    }
}

// ---------------------------------------------------------------- forward, LDS ring
// Forward product with the operands streamed straight into a ring of RING
// K steps in LDS by direct-to-LDS loads (global_load_lds_dwordx4: each lane
// moves 16 bytes to ring base + 16 x lane), so that RING - 1 steps are in
// flight without holding registers.  4 NH wavefronts = 4 row groups x NH
// halves of 32 NH right-hand sides; 5 blocks of 32 rows per wavefront (640
// rows: all sensors of a 600-sensor tile, so the right-hand sides are read
// once per K chunk).  A step is 16 complex columns.
//   A: 640 rows x 64 bytes, rows packed (a load instruction fills 16 rows);
//      the 16-byte chunk c of row r sits in slot c ^ ((r / 4) mod 4), so that
//      16 lanes reading one chunk of 16 consecutive rows hit distinct banks.
//   B: right-hand side b's 128 bytes of the step (4 groups x hi/lo) as 8
//      16-byte parts, part p in slot p ^ ((b / 2) mod 8), so that a load
//      instruction moves 8 whole 128-byte lines (8 right-hand sides) and
//      the 16 lanes of a fragment read (consecutive b) hit distinct banks.
// The K range is rounded up to whole steps; that stays inside the row pitch
// (a multiple of 32 entries >= Nm), where spectrum and right-hand sides
// are zero past Nm, so no step needs masking.
constexpr int kRingSteps = 3;

// Wait until at most n vector-memory loads of this wavefront are in flight
// and its LDS operations are done (expcnt not waited on).
template <int n>
__device__ __forceinline__ void wait_vm_lgkm0() {
    static_assert(n >= 0 && n < 64, "vmcnt field");
    __builtin_amdgcn_s_waitcnt((n & 0xF) | (0x7 << 4) | (0x0 << 8) | ((n >> 4) << 14));
}

// Barrier without a memory fence (the fence would wait for every load in
// flight); the caller's waits make the LDS contents visible.
__device__ __forceinline__ void bare_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// LDS byte address of a shared-memory location.
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// One direct-to-LDS load: 16 bytes per lane from base + off (base
// wavefront-uniform, off a per-lane 32-bit byte offset) to LDS byte address
// lds + 16 x lane (lds wavefront-uniform).  Inline assembly, so that the
// compiler does not wait for it before every LDS access; the kernel waits
// for these loads itself.
__device__ __forceinline__ void dma16(const uint8_t* base, uint32_t off, uint32_t lds) {
    asm volatile("global_load_lds_dwordx4 %0, %1" : : "v"(off), "s"(base), "{m0}"(lds) : "memory");
}
// The same load marked non-temporal, for the spectrum: each of its bytes is
// read once per launch, so its lines need not displace the right-hand sides'
// (measured on load-only rings over a 16.6 GB spectrum: 6.5 -> 7.0 TB/s with
// the adjoint's 2 KB row pieces, 6.1 -> 6.8 TB/s with the whole-line forward
// ring's 128-byte ones).
__device__ __forceinline__ void dma16_stream(const uint8_t* base, uint32_t off, uint32_t lds) {
    asm volatile("global_load_lds_dwordx4 %0, %1 nt" : : "v"(off), "s"(base), "{m0}"(lds) : "memory");
}

// F16: the spectrum is stored in FP16 and the right-hand sides in complex
// FP32 with per-right-hand-side scales (rhs_scale); fragments are rounded to
// FP16 in registers and take one FP16 product per form.
// RG row groups x MB blocks of 32 rows (640 rows: all sensors of a 600-sensor
// operator; 64 or 128 rows for operators with few sensors, where a 640-row
// tile would do the matrix work of its padding rows).
template <int RG, int MB, int NH, bool F16>
__global__ __launch_bounds__(64 * RG * NH) __attribute__((amdgpu_waves_per_eu(NH)))
void k_gemm_fwd_ring(const uint8_t* fhat, const float* __restrict__ scales, const uint8_t* Bq,
                     float2* __restrict__ out_base, GemmArgs ga) {
    constexpr int KU = 2, RING = kRingSteps;
    constexpr int MROWS = RG * 32 * MB, RHS = 32 * NH, NW = RG * NH;
    constexpr int AI = MROWS / 16 / NW;                   // A loads (16 rows each) per wavefront per step
    static_assert(AI >= 1 && AI * 16 * NW == MROWS, "A rows per wavefront");
    constexpr int A_STEP = MROWS * 64;                    // bytes of A per step
    constexpr int B_STEP = RHS * 128;                     // bytes of B per step (8 right-hand sides per load)
    constexpr int BI = RHS / 8 / NW;                      // B loads per wavefront per step
    static_assert(BI >= 1 && 8 * BI * NW == RHS, "B loads per wavefront");
    constexpr int G = AI + BI;                            // loads per wavefront per step
    __shared__ __align__(16) uint8_t ring_a[RING][A_STEP];
    __shared__ __align__(16) uint8_t ring_b[RING][B_STEP];

    const int q = xcd_item(blockIdx.x, ga.Q);
    if (q >= ga.items) return;
    int t = q;
    const int mt = t % ga.n_mt; t /= ga.n_mt;
    const int bg = t % ga.n_bg; t /= ga.n_bg;
    const int kc = t % ga.n_kc; t /= ga.n_kc;
    const int w = t;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rg = wave % RG, nh = wave / RG;
    const int r = lane & 31, kg = lane >> 5;
    const int b0 = bg * RHS;
    const int nb_valid = min(RHS, ga.nrhs - b0);
    const int m0 = mt * MROWS;
    const int kbeg = kc * ga.kchunk;
    const int kend = min((ga.ncols + 15) / 16 * 16, kbeg + ga.kchunk);
    const int nst = (kend - kbeg) / 16;

    // Per-lane byte offsets from wavefront-uniform bases that advance by a
    // step (64 bytes of spectrum row, 128 bytes of right-hand-side row) per
    // step; the launcher checks that the offsets fit 32 bits.  A instruction
    // i of this wavefront fills rows 16 (AI wave + i) .. + 15; lane L takes
    // row L / 4 of those and puts chunk (L % 4) ^ (L / 16 % 4) of it in its
    // slot.
    const uint8_t* const abase = fhat + ((long long)w * ga.Nd * ga.pitch + kbeg) * 4;
    uint32_t aoff[AI];
    {
        const int swz = (lane >> 4) & 3, c = (lane & 3) ^ swz;
#pragma unroll
        for (int i = 0; i < AI; ++i) {
            const int row = 16 * (AI * wave + i) + (lane >> 2);
            const int sr = min(m0 + row, ga.Nd - 1);
            aoff[i] = ((uint32_t)sr * (uint32_t)ga.pitch + 4u * (uint32_t)c) * 4u;
        }
    }
    // B instruction i of this wavefront: right-hand sides 8 (BI wave + i) .. + 7
    // of the group; lane L moves part (L % 8) ^ ((b / 2) mod 8) of right-hand
    // side b = 8 (BI wave + i) + L / 8 into slot L % 8 of its 128 bytes
    const uint8_t* const bbase = Bq + ((long long)w * ga.nrhs + b0) * ga.ldb * 8 + (long long)kbeg * 8;
    uint32_t boff[BI];
#pragma unroll
    for (int i = 0; i < BI; ++i) {
        const int b = 8 * (BI * wave + i) + (lane >> 3);
        const int part = (lane & 7) ^ ((b >> 1) & 7);
        boff[i] = (uint32_t)min(b, nb_valid - 1) * (uint32_t)ga.ldb * 8u + (uint32_t)part * 16u;
    }
    const uint32_t la = lds_addr(&ring_a[0][0]) + AI * wave * 1024, lb = lds_addr(&ring_b[0][0]) + BI * wave * 1024;
    auto issue = [&](int st, int slot) {
        const long long sa = st < nst ? st : nst - 1;       // past the end: repeat the last step (unused)
        const uint8_t* const ab = abase + sa * 64;
#pragma unroll
        for (int i = 0; i < AI; ++i) dma16(ab, aoff[i], la + slot * A_STEP + i * 1024);
#pragma unroll
        for (int i = 0; i < BI; ++i) dma16(bbase + sa * 128, boff[i], lb + slot * B_STEP + i * 1024);
    };

    f32x16 accr[MB], acci[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) accr[mb] = acci[mb] = f32x16{};

    struct Frags {
        uint4 a[MB], bh, bl;
    };
    auto read = [&](Frags& f, int slot, int u) {
        // right-hand side 32 nh + r, group 2 u + kg: parts 2 (2 u + kg) (hi) and + 1 (lo)
        const int rb = 32 * nh + r, sw = (rb >> 1) & 7, ph = 2 * (2 * u + kg);
        f.bh = *reinterpret_cast<const uint4*>(&ring_b[slot][rb * 128 + ((ph ^ sw) * 16)]);
        f.bl = *reinterpret_cast<const uint4*>(&ring_b[slot][rb * 128 + (((ph + 1) ^ sw) * 16)]);
        const int cs = ((2 * u + kg) ^ ((r >> 2) & 3)) * 16;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
            f.a[mb] = *reinterpret_cast<const uint4*>(&ring_a[slot][((rg * MB + mb) * 32 + r) * 64 + cs]);
    };
    // FP16: this lane's right-hand side 32 nh + r (its B fragments, and its outputs)
    float rs = 1.f;
    if constexpr (F16) rs = ga.rhs_scale[min(b0 + 32 * nh + r, ga.nrhs - 1)];
    auto mfmas = [&](const Frags& f) {
        if constexpr (F16) {
            // parts ph and ph + 1 hold entries 4 g .. 4 g + 3 as complex FP32
            const uint4 bx = f_rhs_f16(f.bh, f.bl, rs);
            const uint4 b_r = f_conj(bx), b_i = f_swap(bx);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                accr[mb] = mfma32h(f.a[mb], b_r, accr[mb]);
                acci[mb] = mfma32h(f.a[mb], b_i, acci[mb]);
            }
        } else {
            const uint4 bh_r = f_conj(f.bh), bh_i = f_swap(f.bh), bl_r = f_conj(f.bl), bl_i = f_swap(f.bl);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                accr[mb] = mfma32(f.a[mb], bh_r, accr[mb]);
                acci[mb] = mfma32(f.a[mb], bh_i, acci[mb]);
                accr[mb] = mfma32(f.a[mb], bl_r, accr[mb]);
                acci[mb] = mfma32(f.a[mb], bl_i, acci[mb]);
            }
        }
    };

    // Step st: wait for its loads (RING - 2 later steps stay in flight) and
    // for this wavefront's LDS reads; barrier (every wavefront's loads of
    // step st have landed, every wavefront is done with step st - 1); read
    // the first substep's fragments, so that the matrix cores start as soon
    // as the LDS answers; load step st + RING - 1 into the slot step st - 1
    // used; compute step st.
#pragma unroll
    for (int d = 0; d < RING - 1; ++d) issue(d, d);
    int slot = 0;
    for (int st = 0; st < nst; ++st) {
        wait_vm_lgkm0<(RING - 2) * G>();
        bare_barrier();
        Frags f;
        read(f, slot, 0);
        const int ns = slot == 0 ? RING - 1 : slot - 1;
        issue(st + RING - 1, ns);
        mfmas(f);
#pragma unroll
        for (int u = 1; u < KU; ++u) {
            read(f, slot, u);
            mfmas(f);
        }
        slot = slot + 1 == RING ? 0 : slot + 1;
    }
    wait_vm_lgkm0<0>();                                   // no load may land after the workgroup ends

    const int b = b0 + 32 * nh + r;
    if (b >= ga.nrhs) return;
    const float sc = scales[(long long)w * ga.nblk + kbeg / kScaleBlock] / rs;
    float2* out = out_base + (long long)kc * ga.part_stride + ((long long)w * ga.nrhs + b) * ga.Nd;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = m0 + (rg * MB + mb) * 32 + 8 * (v >> 2) + 4 * kg + (v & 3);
            if (row < ga.Nd) out[row] = make_float2(accr[mb][v] * sc, acci[mb][v] * sc);
        }
}

// ---------------------------------------------------------------- forward, LDS ring, whole lines
// Forward product as in k_gemm_fwd_ring, with steps of 32 complex columns:
// each spectrum row contributes one whole 128-byte line per step (with
// 16-column steps a row gives half a line, and streaming half lines from
// many rows runs well below the rate of whole ones).  RG row groups x MB
// blocks of 32 rows (320 rows for RG = 2, MB = 5: two tiles cover 600
// sensors) x NH halves of 32 NH right-hand sides; four substeps per step.
//   A: MROWS rows x 128 bytes in a 3-step ring; a load instruction fills 8
//      rows; the 16-byte chunk c of row r sits in slot c ^ ((r / 2) mod 8),
//      so that 16 lanes reading one chunk of 16 consecutive rows hit 16
//      distinct bank groups.
//   B: right-hand side b's 256 bytes of the step (8 groups x 2 parts) in a
//      2-step ring, part p in slot p ^ (b mod 16); a load instruction moves
//      4 right-hand sides.  B of step st + 1 is issued before A of step
//      st + 2, so waiting for all but the last step's A loads covers both
//      operands of the next step.
template <int RG, int MB, int NH, bool F16, bool BH>
__global__ __launch_bounds__(64 * RG * NH) __attribute__((amdgpu_waves_per_eu(1)))
void k_gemm_fwd_ring2(const uint8_t* fhat, const float* __restrict__ scales, const uint8_t* Bq,
                      float2* __restrict__ out_base, GemmArgs ga) {
    constexpr int KU = 4;
    constexpr int MROWS = RG * 32 * MB, RHS = 32 * NH, NW = RG * NH;
    constexpr int AI = MROWS / 8 / NW;                    // A loads (8 rows each) per wavefront per step
    static_assert(AI >= 1 && AI * 8 * NW == MROWS, "A rows per wavefront");
    // B bytes per right-hand side and step: 32 complex FP32 (or, BH, FP16 pairs)
    constexpr int BRB = BH ? 128 : 256;
    constexpr int BPI = 1024 / BRB;                       // right-hand sides per B load instruction
    constexpr int BI = RHS / BPI / NW;                    // B loads per wavefront per step
    static_assert(BI >= 1 && BPI * BI * NW == RHS, "B loads per wavefront");
    static_assert(!BH || F16, "FP16 right-hand sides meet an FP16 spectrum");
    constexpr int A_STEP = MROWS * 128, B_STEP = RHS * BRB;
    __shared__ __align__(16) uint8_t ring_a[3][A_STEP];
    __shared__ __align__(16) uint8_t ring_b[2][B_STEP];

    const int q = xcd_item(blockIdx.x, ga.Q);
    if (q >= ga.items) return;
    int t = q;
    const int mt = t % ga.n_mt; t /= ga.n_mt;
    const int bg = t % ga.n_bg; t /= ga.n_bg;
    const int kc = t % ga.n_kc; t /= ga.n_kc;
    const int w = t;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rg = wave % RG, nh = wave / RG;
    const int r = lane & 31, kg = lane >> 5;
    const int b0 = bg * RHS;
    const int nb_valid = min(RHS, ga.nrhs - b0);
    const int m0 = mt * MROWS;
    const int kbeg = kc * ga.kchunk;
    const int kend = min((ga.ncols + 31) / 32 * 32, kbeg + ga.kchunk);
    const int nst = (kend - kbeg) / 32;

    // A instruction i of this wavefront fills tile rows 8 (AI wave + i) ..
    // + 7; lane L takes row L / 8 of those and loads its chunk
    // (L % 8) ^ ((row / 2) mod 8) into slot L % 8.
    const uint8_t* const abase = fhat + ((long long)w * ga.Nd * ga.pitch + kbeg) * 4;
    uint32_t aoff[AI];
#pragma unroll
    for (int i = 0; i < AI; ++i) {
        const int row = 8 * (AI * wave + i) + (lane >> 3);
        const int c = (lane & 7) ^ ((row >> 1) & 7);
        const int sr = min(m0 + row, ga.Nd - 1);
        aoff[i] = ((uint32_t)sr * (uint32_t)ga.pitch) * 4u + 16u * (uint32_t)c;
    }
    // B instruction i: right-hand sides 4 (BI wave + i) .. + 3; lane L moves
    // part (L % 16) ^ (b mod 16) of b = 4 (BI wave + i) + L / 16 into slot L % 16.
    // BH: right-hand sides 8 (BI wave + i) .. + 7, part (L % 8) ^ ((b / 2) mod 8)
    // of b = 8 (BI wave + i) + L / 8 into slot L % 8.
    constexpr uint32_t EB = BH ? 4u : 8u;                 // bytes per complex right-hand-side value
    const uint8_t* const bbase = Bq + ((long long)w * ga.nrhs + b0) * ga.ldb * EB + (long long)kbeg * EB;
    uint32_t boff[BI];
#pragma unroll
    for (int i = 0; i < BI; ++i) {
        const int b = BH ? 8 * (BI * wave + i) + (lane >> 3) : 4 * (BI * wave + i) + (lane >> 4);
        const int part = BH ? (lane & 7) ^ ((b >> 1) & 7) : (lane & 15) ^ (b & 15);
        boff[i] = (uint32_t)min(b, nb_valid - 1) * (uint32_t)ga.ldb * EB + (uint32_t)part * 16u;
    }
    const uint32_t la = lds_addr(&ring_a[0][0]) + AI * wave * 1024, lb = lds_addr(&ring_b[0][0]) + BI * wave * 1024;
    auto issue_a = [&](int st, int slot) {
        const long long sa = st < nst ? st : nst - 1;       // past the end: repeat the last step (unused)
#pragma unroll
        for (int i = 0; i < AI; ++i) dma16_stream(abase + sa * 128, aoff[i], la + slot * A_STEP + i * 1024);
    };
    auto issue_b = [&](int st, int slot) {
        const long long sb = st < nst ? st : nst - 1;
#pragma unroll
        for (int i = 0; i < BI; ++i) dma16(bbase + sb * BRB, boff[i], lb + slot * B_STEP + i * 1024);
    };

    f32x16 accr[MB], acci[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) accr[mb] = acci[mb] = f32x16{};

    struct Frags {
        uint4 a[MB], bh, bl;
    };
    const int rb = 32 * nh + r;
    auto read = [&](Frags& f, int as, int bs, int u) {
        const int g = 2 * u + kg;                         // this lane's group of 4 entries in the step
        if constexpr (BH) {
            f.bh = *reinterpret_cast<const uint4*>(&ring_b[bs][rb * 128 + ((g ^ ((rb >> 1) & 7)) * 16)]);
        } else {
            f.bh = *reinterpret_cast<const uint4*>(&ring_b[bs][rb * 256 + (((2 * g) ^ (rb & 15)) * 16)]);
            f.bl = *reinterpret_cast<const uint4*>(&ring_b[bs][rb * 256 + (((2 * g + 1) ^ (rb & 15)) * 16)]);
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int row = (rg * MB + mb) * 32 + r;
            f.a[mb] = *reinterpret_cast<const uint4*>(&ring_a[as][row * 128 + ((g ^ ((row >> 1) & 7)) * 16)]);
        }
    };
    float rs = 1.f;
    if constexpr (F16) rs = ga.rhs_scale[min(b0 + rb, ga.nrhs - 1)];
    auto mfmas = [&](const Frags& f) {
        if constexpr (F16) {
            const uint4 bx = BH ? f.bh : f_rhs_f16(f.bh, f.bl, rs);
            const uint4 b_r = f_conj(bx), b_i = f_swap(bx);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                accr[mb] = mfma32h(f.a[mb], b_r, accr[mb]);
                acci[mb] = mfma32h(f.a[mb], b_i, acci[mb]);
            }
        } else {
            const uint4 bh_r = f_conj(f.bh), bh_i = f_swap(f.bh), bl_r = f_conj(f.bl), bl_i = f_swap(f.bl);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                accr[mb] = mfma32(f.a[mb], bh_r, accr[mb]);
                acci[mb] = mfma32(f.a[mb], bh_i, acci[mb]);
                accr[mb] = mfma32(f.a[mb], bl_r, accr[mb]);
                acci[mb] = mfma32(f.a[mb], bl_i, acci[mb]);
            }
        }
    };

    // Issue order B_0, A_0, A_1, then per step st: B_{st+1}, A_{st+2}.  At
    // step st, waiting until at most AI loads are in flight leaves only
    // A_{st+1} outstanding: A_st and B_st have landed.
    issue_b(0, 0);
    issue_a(0, 0);
    issue_a(1, 1);
    int as = 0, bs = 0;
    for (int st = 0; st < nst; ++st) {
        wait_vm_lgkm0<AI>();
        bare_barrier();
        Frags f;
        read(f, as, bs, 0);
        issue_b(st + 1, bs ^ 1);                          // the slot step st - 1 used
        issue_a(st + 2, as == 0 ? 2 : as - 1);            // the slot step st - 1 used
        mfmas(f);
#pragma unroll
        for (int u = 1; u < KU; ++u) {
            read(f, as, bs, u);
            mfmas(f);
        }
        as = as == 2 ? 0 : as + 1;
        bs ^= 1;
    }
    wait_vm_lgkm0<0>();                                   // no load may land after the workgroup ends

    // Partial products, a half of the right-hand sides at a time, through
    // the spectrum ring: the half's wavefronts write their scaled
    // accumulators as [right-hand side][row] rows (OS_RS bytes apart), then
    // the workgroup stores whole rows, 16 bytes per lane, non-temporal (the
    // accumulator layout gives 8-byte pieces spread over 32 rows).
    constexpr int OS_RS = MROWS * 8 + 16;
    static_assert(32 * OS_RS <= 3 * A_STEP, "a half's products fit the spectrum ring");
    uint8_t* const stg = &ring_a[0][0];
    const float sc = scales[(long long)w * ga.nblk + kbeg / kScaleBlock] / rs;
    float2* const out_w = out_base + (long long)kc * ga.part_stride + (long long)w * ga.nrhs * ga.Nd;
    const bool pairs = (ga.Nd & 1) == 0;                  // rows of even length: 16-byte aligned pairs
    constexpr int CPR = MROWS / 2;                        // pairs per staged row
#pragma unroll 1
    for (int h = 0; h < NH; ++h) {
        bare_barrier();                                   // ring reads (or the previous half's) done
        if (nh == h) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int row = (rg * MB + mb) * 32 + 8 * (v >> 2) + 4 * kg + (v & 3);
                    *reinterpret_cast<float2*>(&stg[r * OS_RS + row * 8]) =
                        make_float2(accr[mb][v] * sc, acci[mb][v] * sc);
                }
        }
        wait_vm_lgkm0<63>();                              // this wavefront's LDS writes done
        bare_barrier();
        for (int e = tid; e < 32 * CPR; e += 64 * NW) {
            const int rr = e / CPR, c = 2 * (e - rr * CPR);
            const int b = b0 + 32 * h + rr, row = m0 + c;
            if (b < ga.nrhs && row < ga.Nd) {
                const float4 v = *reinterpret_cast<const float4*>(&stg[rr * OS_RS + c * 8]);
                float2* o = out_w + (long long)b * ga.Nd + row;
                if (pairs && row + 1 < ga.Nd) {
                    store_nt(reinterpret_cast<float4*>(o), v);
                } else {
                    o[0] = make_float2(v.x, v.y);
                    if (row + 1 < ga.Nd) o[1] = make_float2(v.z, v.w);
                }
            }
        }
    }
}

// ---------------------------------------------------------------- adjoint, LDS ring
// Adjoint product with both operands streamed into a RING-step LDS ring by
// direct-to-LDS loads, as in the forward ring.  RG NH wavefronts = RG column
// groups x NH halves of 32 NH right-hand sides; MB blocks of 32 output
// columns per wavefront (MROWS = 32 RG MB columns per workgroup).  A step is
// 16 sensors (two substeps of 8).
//   A: 16 sensor rows x MROWS columns; a load instruction moves 256 columns
//      of one row (1 KB, whole lines); rows A_RS = 4 MROWS + 32 bytes apart,
//      so the two sensor quartets a fragment gathers (rows 4 apart) fall in
//      different halves of the 64 banks.
//   B: as in the forward ring, right-hand side b's 128 bytes of the step
//      (4 sensor groups x hi/lo) in 8 parts, part p in slot p ^ ((b / 2) mod 8).
// The data rows are padded with zeros to a multiple of 16 sensors (ldb), so
// every step is whole; sensor rows past Nd read row Nd - 1 and columns past
// the pitch read its last entries (valid addresses), and a substep that
// starts at or past Nd is skipped (its data rows are zero).
template <int RG, int MB, int NH, bool F16>
__global__ __launch_bounds__(64 * RG * NH) __attribute__((amdgpu_waves_per_eu(2)))
void k_gemm_adj_ring(const uint8_t* fhat, const float* __restrict__ scales, const uint8_t* Bq,
                     float2* __restrict__ out_base, GemmArgs ga) {
    constexpr int KU = 2, RING = kRingSteps, NW = RG * NH;
    constexpr int MROWS = 32 * RG * MB, RHS = 32 * NH;
    constexpr int NCP = MROWS / 256;                      // load instructions per sensor row
    constexpr int AI = 16 * NCP / NW;                     // A loads per wavefront per step
    constexpr int BI = RHS / 8 / NW;                      // B loads (8 right-hand sides each) per wavefront per step
    static_assert(MROWS % 256 == 0 && AI * NW == 16 * NCP && BI * 8 * NW == RHS, "loads per wavefront");
    constexpr int A_RS = 4 * MROWS + 32;
    constexpr int A_STEP = 16 * A_RS;
    constexpr int B_STEP = RHS * 128;
    constexpr int G = AI + BI;
    // Output staging (after the K loop, over the ring): 32 right-hand sides x
    // CW columns of complex FP32 at a time (CW: MROWS or the largest part of
    // it that fits, in whole wavefront column ranges), rows OS_RS bytes apart
    // (16 bytes of padding shift consecutive rows across the banks).
    constexpr int LDS_BYTES = RING * (A_STEP + B_STEP);
    constexpr int CW = 32 * (MROWS * 8 + 16) <= LDS_BYTES       ? MROWS
                       : 32 * (MROWS / 2 * 8 + 16) <= LDS_BYTES ? MROWS / 2
                                                                : MROWS / 4;
    constexpr int OS_RS = CW * 8 + 16;
    constexpr bool STAGE = 32 * OS_RS <= LDS_BYTES && CW % (32 * MB) == 0;
    __shared__ __align__(16) uint8_t lds[LDS_BYTES];
    uint8_t (*ring_a)[A_STEP] = reinterpret_cast<uint8_t (*)[A_STEP]>(lds);
    uint8_t (*ring_b)[B_STEP] = reinterpret_cast<uint8_t (*)[B_STEP]>(lds + RING * A_STEP);

    const int q = xcd_item(blockIdx.x, ga.Q);
    if (q >= ga.items) return;
    int t = q;
    const int mt = t % ga.n_mt; t /= ga.n_mt;
    const int bg = t % ga.n_bg; t /= ga.n_bg;
    const int w = t;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rg = wave % RG, nh = wave / RG;
    const int r = lane & 31, kg = lane >> 5;
    const int b0 = bg * RHS;
    const int nb_valid = min(RHS, ga.nrhs - b0);
    const int m0 = mt * MROWS;                            // first output column of the tile
    const int nst = ga.ldb / 16;                          // ldb is a multiple of 16

    // A instruction i of this wavefront: sensor row k = a / NCP of the step,
    // columns m0 + 256 (a % NCP) + 4 lane .. + 3 (a = AI wave + i)
    const uint8_t* const arows = fhat + (long long)w * ga.Nd * ga.pitch * 4;
    uint32_t aoff[AI];
#pragma unroll
    for (int i = 0; i < AI; ++i) {
        const int a = AI * wave + i;
        aoff[i] = (uint32_t)min(m0 + 256 * (a % NCP) + 4 * lane, ga.pitch - 4) * 4u;
    }
    // B instruction i: right-hand sides 8 (BI wave + i) .. + 7, lane L
    // moving part (L % 8) ^ ((b / 2) mod 8) of b = 8 (BI wave + i) + L / 8
    const uint8_t* const brows = Bq + ((long long)w * ga.nrhs + b0) * ga.ldb * 8;
    uint32_t boff[BI];
#pragma unroll
    for (int i = 0; i < BI; ++i) {
        const int b = 8 * (BI * wave + i) + (lane >> 3);
        const int part = (lane & 7) ^ ((b >> 1) & 7);
        boff[i] = (uint32_t)min(b, nb_valid - 1) * (uint32_t)ga.ldb * 8u + (uint32_t)part * 16u;
    }
    const uint32_t la = lds_addr(&ring_a[0][0]), lb = lds_addr(&ring_b[0][0]) + BI * wave * 1024;
    auto issue = [&](int st, int slot) {
        const int sa = st < nst ? st : nst - 1;           // past the end: repeat the last step (unused)
#pragma unroll
        for (int i = 0; i < AI; ++i) {
            const int a = AI * wave + i, k = a / NCP;
            const int row = min(16 * sa + k, ga.Nd - 1);
            dma16_stream(arows + (long long)row * ga.pitch * 4, aoff[i], la + slot * A_STEP + k * A_RS + (a % NCP) * 1024);
        }
#pragma unroll
        for (int i = 0; i < BI; ++i) dma16(brows + (long long)sa * 128, boff[i], lb + slot * B_STEP + i * 1024);
    };

    f32x16 accr[MB], acci[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) accr[mb] = acci[mb] = f32x16{};

    // lane (r, kg) of block mb, substep u: sensors 8 u + 4 kg .. + 3 of the
    // step for column (rg MB + mb) 32 + r
    struct Frags {
        uint4 a[MB], bh, bl;
    };
    auto read = [&](Frags& f, int slot, int u) {
        // right-hand side 32 nh + r, group 2 u + kg: parts 2 (2 u + kg) (hi) and + 1 (lo)
        const int rb = 32 * nh + r, sw = (rb >> 1) & 7, ph = 2 * (2 * u + kg);
        f.bh = *reinterpret_cast<const uint4*>(&ring_b[slot][rb * 128 + ((ph ^ sw) * 16)]);
        f.bl = *reinterpret_cast<const uint4*>(&ring_b[slot][rb * 128 + (((ph + 1) ^ sw) * 16)]);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const uint8_t* p = &ring_a[slot][(8 * u + 4 * kg) * A_RS + ((rg * MB + mb) * 32 + r) * 4];
            f.a[mb] = make_uint4(*reinterpret_cast<const uint32_t*>(p), *reinterpret_cast<const uint32_t*>(p + A_RS),
                                 *reinterpret_cast<const uint32_t*>(p + 2 * A_RS),
                                 *reinterpret_cast<const uint32_t*>(p + 3 * A_RS));
        }
    };
    // FP16: this lane's right-hand side 32 nh + r (its B fragments, and its outputs)
    float rs = 1.f;
    if constexpr (F16) rs = ga.rhs_scale[min(b0 + 32 * nh + r, ga.nrhs - 1)];
    auto mfmas = [&](const Frags& f) {
        if constexpr (F16) {
            const uint4 bx = f_rhs_f16(f.bh, f.bl, rs);
            const uint4 b_i = f_nswap(bx);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                accr[mb] = mfma32h(f.a[mb], bx, accr[mb]);
                acci[mb] = mfma32h(f.a[mb], b_i, acci[mb]);
            }
        } else {
            const uint4 bh_i = f_nswap(f.bh), bl_i = f_nswap(f.bl);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                accr[mb] = mfma32(f.a[mb], f.bh, accr[mb]);
                acci[mb] = mfma32(f.a[mb], bh_i, acci[mb]);
                accr[mb] = mfma32(f.a[mb], f.bl, accr[mb]);
                acci[mb] = mfma32(f.a[mb], bl_i, acci[mb]);
            }
        }
    };
    const float irs = 1.f / rs;                           // exact: rs is a power of two

#pragma unroll
    for (int d = 0; d < RING - 1; ++d) issue(d, d);
    int slot = 0;
    for (int st = 0; st < nst; ++st) {
        wait_vm_lgkm0<(RING - 2) * G>();
        bare_barrier();
        Frags f;
        read(f, slot, 0);                                 // first fragments before the next loads
        const int ns = slot == 0 ? RING - 1 : slot - 1;
        issue(st + RING - 1, ns);
        mfmas(f);
        if (16 * st + 8 < ga.Nd) {
            read(f, slot, 1);
            mfmas(f);
        }
        slot = slot + 1 == RING ? 0 : slot + 1;
    }
    wait_vm_lgkm0<0>();                                   // no load may land after the workgroup ends

    if constexpr (STAGE) {
        // Each (half of the right-hand sides, column part) in turn: its
        // wavefronts write their scaled products to LDS, then the whole
        // workgroup stores rows of CW columns (16 bytes per lane, whole lines)
        // instead of the accumulators' 8-byte pieces spread over 32 rows.
        for (int ch = 0; ch < NH * (MROWS / CW); ++ch) {
            const int h = ch / (MROWS / CW), c0 = (ch % (MROWS / CW)) * CW;
            bare_barrier();                               // ring (or previous part) reads done
            if (nh == h && rg * MB * 32 / CW == c0 / CW) {
                // FP16 output: this lane's right-hand side's scale folded in here
                const int bo = b0 + 32 * nh + r;
                const float os = F16 && ga.out_scale && bo < ga.nrhs ? ga.out_scale[bo] : 1.f;
#pragma unroll
                for (int mb = 0; mb < MB; ++mb) {
                    const int cb = (rg * MB + mb) * 32;   // an m block lies in one 4096-column scale block
                    const float sc =
                        scales[(long long)w * ga.nblk + min(m0 + cb, ga.ncols - 1) / kScaleBlock] * irs * os;
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const int c = cb - c0 + 8 * (v >> 2) + 4 * kg + (v & 3);
                        *reinterpret_cast<float2*>(&lds[r * OS_RS + c * 8]) =
                            make_float2(accr[mb][v] * sc, acci[mb][v] * sc);
                    }
                }
            }
            __syncthreads();
            constexpr int PER = 64 * NW * 2;              // complex values stored per pass
#pragma unroll 4
            for (int e = tid * 2; e < 32 * CW; e += PER) {
                const int row = e / CW, c = e % CW;
                const int b = b0 + 32 * h + row, j = m0 + c0 + c;
                const float4 v = *reinterpret_cast<const float4*>(&lds[row * OS_RS + c * 8]);
                if (b < ga.nrhs && j < ga.ncols) {
                    const long long at = ((long long)w * ga.nrhs + b) * ga.pitch + j;
                    if (F16 && ga.out_scale) {
                        // FP16 pairs (already scaled): the same index in a 4-byte array
                        uint32_t* o = reinterpret_cast<uint32_t*>(out_base) + at;
                        if (j + 1 < ga.ncols)
                            store_nt(reinterpret_cast<uint2*>(o), make_uint2(pack_f16(v.x, v.y, 1.f), pack_f16(v.z, v.w, 1.f)));
                        else
                            store_nt(o, pack_f16(v.x, v.y, 1.f));
                    } else {
                        float2* o = out_base + at;
                        if (j + 1 < ga.ncols)
                            store_nt(reinterpret_cast<float4*>(o), v);
                        else
                            store_nt(o, make_float2(v.x, v.y));
                    }
                }
            }
        }
    } else {
        const int b = b0 + 32 * nh + r;
        if (b >= ga.nrhs) return;
        float2* out = out_base + ((long long)w * ga.nrhs + b) * ga.pitch;
        uint32_t* outh = reinterpret_cast<uint32_t*>(out_base) + ((long long)w * ga.nrhs + b) * ga.pitch;
        const float os = F16 && ga.out_scale ? ga.out_scale[b] : 0.f;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int jb = m0 + (rg * MB + mb) * 32;        // an m block lies in one 4096-column scale block
            if (jb >= ga.ncols) continue;
            const float sc = scales[(long long)w * ga.nblk + jb / kScaleBlock] * irs;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int j = jb + 8 * (v >> 2) + 4 * kg + (v & 3);
                if (j < ga.ncols) {
                    if (F16 && ga.out_scale)
                        outh[j] = pack_f16(accr[mb][v] * sc, acci[mb][v] * sc, os);
                    else
                        out[j] = make_float2(accr[mb][v] * sc, acci[mb][v] * sc);
                }
            }
        }
    }
}

// Scales of the FP16 operands of a data-space column call, per right-hand
// side b, from the adjoint's input: every adjoint product of b satisfies
// |sum_s conj(F_w[s, j]) y_w[s]| <= B = max_w (2^15 m_w sum_s (|re y| + |im y|)),
// m_w the largest multiplier of frequency w's stored spectrum (stored values
// are at most 2^15 in magnitude), and the truncate-and-repad maps a spectrum
// bounded by B to one bounded by Nt B (each time value is at most B, each
// output bin a sum of Nt of them).  sx[b] = the largest power of two with
// B sx <= 2^14 (the adjoint's FP16 outputs), sy[b] the same for Nt B (the
// re-padded FP16 right-hand sides of the forward products); 1 when B = 0.
// First pass: a wavefront per (frequency, right-hand side) row writes
// m_w sum_s (|re y| + |im y|) to part; second pass: the maximum over the
// frequencies, one wavefront per right-hand side.
__device__ __forceinline__ float pow2_at_most(float x) {
    if (!(x > 0.f) || !(x < 3.0e38f)) return 1.f;
    int e;
    frexpf(x, &e);                                       // x = f 2^e, f in [1/2, 1)
    return ldexpf(1.f, max(-126, min(126, e - 1)));
}

__global__ __launch_bounds__(1024) void k_fp16_operand_rows(const float2* __restrict__ Y, int ld, int nrhs, int nfreq,
                                                            int Nd, const float* __restrict__ scales, int nblk,
                                                            float* __restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * 16 + (threadIdx.x >> 6);          // w nrhs + b
    if (row >= nfreq * nrhs) return;
    const int w = row / nrhs;
    const float2* y = Y + (long long)row * ld;
    float t = 0.f;
    for (int s = lane; s < Nd; s += 64) {
        const float2 v = y[s];
        t += fabsf(v.x) + fabsf(v.y);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    if (lane == 0) {
        float m = 0.f;
        for (int k = 0; k < nblk; ++k) m = fmaxf(m, scales[(long long)w * nblk + k]);
        part[row] = t * m;
    }
}

__global__ __launch_bounds__(64) void k_fp16_operand_scales(const float* __restrict__ part, int nrhs, int nfreq, int Nt,
                                                            float* __restrict__ sx, float* __restrict__ sy) {
    const int b = blockIdx.x;
    float v = 0.f;
    for (int w = threadIdx.x; w < nfreq; w += 64) v = fmaxf(v, part[(long long)w * nrhs + b]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    if (threadIdx.x == 0) {
        const float bound = v * 32768.f;
        sx[b] = bound > 0.f ? pow2_at_most(16384.f / bound) : 1.f;
        sy[b] = bound > 0.f ? pow2_at_most(16384.f / (bound * (float)Nt)) : 1.f;
    }
}

hipError_t launch_fp16_operand_scales(const void* Y, int ld, int nrhs, int nfreq, int Nd, const float* scales, int nblk,
                                      int Nt, float* part, float* sx, float* sy, hipStream_t st) {
    const int rows = nfreq * nrhs;
    hipLaunchKernelGGL(k_fp16_operand_rows, dim3((rows + 15) / 16), dim3(1024), 0, st, (const float2*)Y, ld, nrhs, nfreq,
                       Nd, scales, nblk, part);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_fp16_operand_scales, dim3(nrhs), dim3(64), 0, st, (const float*)part, nrhs, nfreq, Nt, sx, sy);
    return hipGetLastError();
}

// Operand filler for timing runs: words of two BF16 values with magnitudes in
// [1/2, 1) and hashed signs and mantissas.  The matrix cores draw much more
// power on such data than on zeros, and the power limit sets their clock, so
// tiles are compared on data like the real operands.
__global__ void k_fill_bf16(uint32_t* __restrict__ p, size_t n, uint32_t seed) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i * 0x9E3779B1u ^ seed;
        h ^= h >> 15; h *= 0x85EBCA77u; h ^= h >> 13; h *= 0xC2B2AE3Du; h ^= h >> 16;
        const uint32_t a = (h & 0x807Fu) | (126u << 7), b = ((h >> 16) & 0x807Fu) | (126u << 7);
        p[i] = a | (b << 16);
    }
}

hipError_t launch_fill_bf16(void* p, size_t bytes, uint32_t seed, hipStream_t st) {
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_bf16, dim3(2048), dim3(256), 0, st, (uint32_t*)p, n, seed);
    return hipGetLastError();
}

__global__ void k_fill_f32(float* __restrict__ p, size_t n, float v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)std::min<size_t>(1024, (n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------- host launchers
int gemm_fwd_kchunks(int ncols) { return (ncols + kScaleBlock - 1) / kScaleBlock; }

int gemm_data_pitch(int Nd) { return (Nd + 15) / 16 * 16; }

template <bool FWD, int RG, int KU, int MB, int WPE, int PF, int NW = 4>
static hipError_t launch_tile(GemmArgs ga, const void* fhat, const float* scales, const void* Bq, void* out,
                              hipStream_t st) {
    using T = Tile<FWD, RG, KU, MB, NW>;
    ga.n_mt = ((FWD ? ga.Nd : ga.ncols) + T::MROWS - 1) / T::MROWS;
    ga.n_bg = (ga.nrhs + T::RHS - 1) / T::RHS;
    ga.items = ga.nfreq * ga.n_kc * ga.n_bg * ga.n_mt;
    ga.Q = (ga.items + 7) / 8;
    hipLaunchKernelGGL((k_gemm<FWD, RG, KU, MB, WPE, PF, NW>), dim3(8 * ga.Q), dim3(T::THREADS), 0, st, (const uint8_t*)fhat,
                       scales, (const uint8_t*)Bq, (float2*)out, ga);
    return hipGetLastError();
}

// Tile variants (row groups RG, substeps per step KU, 32-row blocks per
// wavefront MB, wavefronts per SIMD WPE, staged steps PF, wavefronts per
// workgroup NW): 32 (NW / RG) right-hand sides and 32 MB RG output rows per
// workgroup, K steps of 8 KU entries.  NW = 8 with RG = 4 covers 600 sensors
// and 64 right-hand sides in one workgroup, so the right-hand sides are read
// once per K chunk instead of once per 320-row tile.  MB = 5 fits
// 600-sensor forward tiles (two of 320 or one of 640 rows); MB = 4 keeps the
// accumulators at 128 registers so that two workgroups share a CU, which
// lets one workgroup's loads run under another's prologue and epilogue (the
// adjoint's 256-column tiles also divide 4096-column blocks evenly).  A
// plan's autotuner may replace the built-in choice (gemm_default_tile).
// Variants 7 and 8 are the forward LDS-ring kernel (k_gemm_fwd_ring, pf = 0
// marks a ring) with 640-row tiles for 64 and 32 right-hand sides per group,
// 11 and 12 the same kernel with 64- and 128-row tiles (64 right-hand sides),
// 13 and 14 the whole-line forward ring (k_gemm_fwd_ring2, 320-row tiles,
// 32-column steps) for 64 and 32, 9 and 10 the adjoint one
// (k_gemm_adj_ring) for 64 and 32, 15 and 16 the adjoint ring with 512
// columns and 64 right-hand sides and with 256 columns and 32, 17 and 18 the
// whole-line forward ring with 64- and 128-row tiles (64 right-hand sides:
// operators with few sensors, also on FP16 right-hand sides); a direction a
// variant lacks takes its built-in choice.
struct TileShape {
    int rg, ku, mb, wpe, pf, nw;
    int dirs;   // 1: forward, 2: adjoint, 3: both
};
static const TileShape kTiles[] = {{2, 4, 5, 1, 2, 4, 3}, {2, 2, 5, 1, 2, 4, 3}, {4, 2, 5, 1, 2, 4, 3},
                                   {2, 2, 4, 2, 2, 4, 3}, {4, 2, 4, 2, 2, 4, 3}, {2, 2, 5, 2, 1, 4, 3},
                                   {4, 2, 5, 2, 1, 8, 3}, {4, 2, 5, 2, 0, 8, 1}, {4, 2, 5, 1, 0, 4, 1},
                                   {2, 2, 4, 2, 0, 4, 2}, {4, 2, 4, 1, 0, 4, 2}, {2, 2, 1, 2, 0, 4, 1},
                                   {4, 2, 1, 2, 0, 8, 1}, {2, 4, 5, 1, 0, 4, 1}, {2, 4, 5, 1, 0, 2, 1},
                                   {4, 2, 4, 1, 0, 8, 2}, {2, 2, 4, 2, 0, 2, 2}, {2, 4, 1, 2, 0, 4, 1},
                                   {4, 4, 1, 2, 0, 8, 1}};
constexpr int kTileCount = sizeof(kTiles) / sizeof(kTiles[0]);

int gemm_tile_count() { return kTileCount; }

bool gemm_tile_has(int tile, bool fwd) {
    return tile >= 0 && tile < kTileCount && (kTiles[tile].dirs & (fwd ? 1 : 2)) != 0;
}

template <int RG, int MB, int NH>
static hipError_t launch_ring(GemmArgs ga, const void* fhat, const float* scales, const void* Bq, void* out,
                              hipStream_t st) {
    // the ring kernel addresses a frequency's spectrum and a group's
    // right-hand-side rows with 32-bit byte offsets; larger shapes take the
    // register-staged 640-row tile
    if ((long long)ga.Nd * ga.pitch * 4 >= (1LL << 32) || 32LL * NH * ga.ldb * 8 >= (1LL << 32)) {
        if (ga.a_f16) return hipErrorInvalidValue;        // callers check gemm_f16_fits first
        return launch_tile<true, 4, 2, 5, 2, 1, 8>(ga, fhat, scales, Bq, out, st);
    }
    constexpr int MROWS = 32 * RG * MB;
    ga.n_mt = (ga.Nd + MROWS - 1) / MROWS;
    ga.n_bg = (ga.nrhs + 32 * NH - 1) / (32 * NH);
    ga.items = ga.nfreq * ga.n_kc * ga.n_bg * ga.n_mt;
    ga.Q = (ga.items + 7) / 8;
    if (ga.a_f16)
        hipLaunchKernelGGL((k_gemm_fwd_ring<RG, MB, NH, true>), dim3(8 * ga.Q), dim3(64 * RG * NH), 0, st,
                           (const uint8_t*)fhat, scales, (const uint8_t*)Bq, (float2*)out, ga);
    else
        hipLaunchKernelGGL((k_gemm_fwd_ring<RG, MB, NH, false>), dim3(8 * ga.Q), dim3(64 * RG * NH), 0, st,
                           (const uint8_t*)fhat, scales, (const uint8_t*)Bq, (float2*)out, ga);
    return hipGetLastError();
}

template <int RG, int MB, int NH>
static hipError_t launch_ring2(GemmArgs ga, const void* fhat, const float* scales, const void* Bq, void* out,
                               hipStream_t st) {
    // 32-bit lane offsets, as in the 16-column ring
    if ((long long)ga.Nd * ga.pitch * 4 >= (1LL << 32) || 32LL * NH * ga.ldb * 8 >= (1LL << 32) || ga.kchunk % 32 ||
        ga.pitch % 32) {
        if (ga.a_f16) return hipErrorInvalidValue;        // callers check gemm_f16_fits first
        return launch_tile<true, 4, 2, 5, 2, 1, 8>(ga, fhat, scales, Bq, out, st);
    }
    constexpr int MROWS = 32 * RG * MB;
    ga.n_mt = (ga.Nd + MROWS - 1) / MROWS;
    ga.n_bg = (ga.nrhs + 32 * NH - 1) / (32 * NH);
    ga.items = ga.nfreq * ga.n_kc * ga.n_bg * ga.n_mt;
    ga.Q = (ga.items + 7) / 8;
    if (ga.a_f16 && ga.b_f16)
        hipLaunchKernelGGL((k_gemm_fwd_ring2<RG, MB, NH, true, true>), dim3(8 * ga.Q), dim3(64 * RG * NH), 0, st,
                           (const uint8_t*)fhat, scales, (const uint8_t*)Bq, (float2*)out, ga);
    else if (ga.a_f16)
        hipLaunchKernelGGL((k_gemm_fwd_ring2<RG, MB, NH, true, false>), dim3(8 * ga.Q), dim3(64 * RG * NH), 0, st,
                           (const uint8_t*)fhat, scales, (const uint8_t*)Bq, (float2*)out, ga);
    else
        hipLaunchKernelGGL((k_gemm_fwd_ring2<RG, MB, NH, false, false>), dim3(8 * ga.Q), dim3(64 * RG * NH), 0, st,
                           (const uint8_t*)fhat, scales, (const uint8_t*)Bq, (float2*)out, ga);
    return hipGetLastError();
}

template <int RG, int MB, int NH>
static hipError_t launch_adj_ring(GemmArgs ga, const void* fhat, const float* scales, const void* Bq, void* out,
                                  hipStream_t st) {
    // 32-bit lane offsets within a spectrum row and a group's right-hand-side rows
    if ((long long)ga.pitch * 4 >= (1LL << 32) || 32LL * NH * ga.ldb * 8 >= (1LL << 32)) {
        if (ga.a_f16) return hipErrorInvalidValue;        // callers check gemm_f16_fits first
        return launch_tile<false, 2, 2, 4, 2, 2>(ga, fhat, scales, Bq, out, st);
    }
    constexpr int MROWS = 32 * RG * MB;
    ga.n_mt = (ga.ncols + MROWS - 1) / MROWS;
    ga.n_bg = (ga.nrhs + 32 * NH - 1) / (32 * NH);
    ga.items = ga.nfreq * ga.n_bg * ga.n_mt;
    ga.Q = (ga.items + 7) / 8;
    if (ga.a_f16)
        hipLaunchKernelGGL((k_gemm_adj_ring<RG, MB, NH, true>), dim3(8 * ga.Q), dim3(64 * RG * NH), 0, st,
                           (const uint8_t*)fhat, scales, (const uint8_t*)Bq, (float2*)out, ga);
    else
        hipLaunchKernelGGL((k_gemm_adj_ring<RG, MB, NH, false>), dim3(8 * ga.Q), dim3(64 * RG * NH), 0, st,
                           (const uint8_t*)fhat, scales, (const uint8_t*)Bq, (float2*)out, ga);
    return hipGetLastError();
}

bool gemm_tile_is_ring(int tile) { return tile >= 0 && tile < kTileCount && kTiles[tile].pf == 0; }

// FP16 spectra run on the LDS-ring kernels only, whose 32-bit lane offsets
// must cover a frequency's spectrum and a group's right-hand-side rows.
bool gemm_f16_fits(int Nd, int pitch) {
    const long long ldb = gemm_data_pitch(Nd);
    return (long long)Nd * pitch * 4 < (1LL << 32) && 64LL * pitch * 8 < (1LL << 32) && 64LL * ldb * 8 < (1LL << 32);
}

int gemm_tile_shape(int tile, int* rg, int* ku, int* mb, int* rhs) {
    if (tile < 0 || tile >= kTileCount) return -1;
    *rg = kTiles[tile].rg;
    *ku = kTiles[tile].ku;
    *mb = kTiles[tile].mb;
    *rhs = 32 * kTiles[tile].nw / kTiles[tile].rg;
    return 0;
}

// Built-in choice without autotuning: the variants measured fastest on the
// 600 x 16384 x 420 workload (random operands) for each width (the LDS
// rings: 7 / 9 above 32 right-hand sides, 8 / 10 for at most 32); forward
// products of operators with at most 64 or 128 sensors take the 64- or
// 128-row ring tiles 11 / 12 (64 right-hand sides per group).
int gemm_default_tile(int nrhs, bool fwd, int Nd) {
    if (fwd && Nd <= 64) return 11;
    if (fwd && Nd <= 128) return 12;
    return nrhs > 32 ? (fwd ? 7 : 9) : (fwd ? 8 : 10);
}

hipError_t launch_gemm_fwd(const GemmArgs& in, int tile, const void* fhat, const float* scales, const void* Xq,
                           void* Yp, hipStream_t st) {
    if (in.a_f16 && !in.rhs_scale) return hipErrorInvalidValue;      // FP16 products read per-RHS scales
    GemmArgs ga = in;
    ga.ldb = ga.pitch;
    ga.kchunk = kScaleBlock;
    ga.n_kc = gemm_fwd_kchunks(ga.ncols);
    if (!gemm_tile_has(tile, true) || (ga.a_f16 && !gemm_tile_is_ring(tile))) tile = gemm_default_tile(ga.nrhs, true, ga.Nd);
    if (ga.b_f16) {                                    // FP16 right-hand sides: the whole-line ring only
        if (!ga.a_f16) return hipErrorInvalidValue;
        tile = ga.Nd <= 64 ? 17 : ga.Nd <= 128 ? 18 : ga.nrhs > 32 ? 13 : 14;
    }
    switch (tile) {
        case 0: return launch_tile<true, 2, 4, 5, 1, 2>(ga, fhat, scales, Xq, Yp, st);
        case 1: return launch_tile<true, 2, 2, 5, 1, 2>(ga, fhat, scales, Xq, Yp, st);
        case 2: return launch_tile<true, 4, 2, 5, 1, 2>(ga, fhat, scales, Xq, Yp, st);
        case 3: return launch_tile<true, 2, 2, 4, 2, 2>(ga, fhat, scales, Xq, Yp, st);
        case 4: return launch_tile<true, 4, 2, 4, 2, 2>(ga, fhat, scales, Xq, Yp, st);
        case 5: return launch_tile<true, 2, 2, 5, 2, 1>(ga, fhat, scales, Xq, Yp, st);
        case 6: return launch_tile<true, 4, 2, 5, 2, 1, 8>(ga, fhat, scales, Xq, Yp, st);
        case 7: return launch_ring<4, 5, 2>(ga, fhat, scales, Xq, Yp, st);
        case 8: return launch_ring<4, 5, 1>(ga, fhat, scales, Xq, Yp, st);
        case 11: return launch_ring<2, 1, 2>(ga, fhat, scales, Xq, Yp, st);
        case 12: return launch_ring<4, 1, 2>(ga, fhat, scales, Xq, Yp, st);
        case 13: return launch_ring2<2, 5, 2>(ga, fhat, scales, Xq, Yp, st);
        case 14: return launch_ring2<2, 5, 1>(ga, fhat, scales, Xq, Yp, st);
        case 17: return launch_ring2<2, 1, 2>(ga, fhat, scales, Xq, Yp, st);
        case 18: return launch_ring2<4, 1, 2>(ga, fhat, scales, Xq, Yp, st);
        default: return launch_tile<true, 4, 2, 5, 2, 1, 8>(ga, fhat, scales, Xq, Yp, st);
    }
}

hipError_t launch_gemm_adj(const GemmArgs& in, int tile, const void* fhat, const float* scales, const void* Yq,
                           void* Xp, hipStream_t st) {
    if (in.a_f16 && !in.rhs_scale) return hipErrorInvalidValue;      // FP16 products read per-RHS scales
    GemmArgs ga = in;
    ga.ldb = gemm_data_pitch(ga.Nd);
    ga.kchunk = 0;
    ga.n_kc = 1;
    if (!gemm_tile_has(tile, false) || (ga.a_f16 && !gemm_tile_is_ring(tile))) tile = gemm_default_tile(ga.nrhs, false, ga.Nd);
    switch (tile) {
        case 0: return launch_tile<false, 2, 4, 5, 1, 2>(ga, fhat, scales, Yq, Xp, st);
        case 1: return launch_tile<false, 2, 2, 5, 1, 2>(ga, fhat, scales, Yq, Xp, st);
        case 2: return launch_tile<false, 4, 2, 5, 1, 2>(ga, fhat, scales, Yq, Xp, st);
        case 3: return launch_tile<false, 2, 2, 4, 2, 2>(ga, fhat, scales, Yq, Xp, st);
        case 4: return launch_tile<false, 4, 2, 4, 2, 2>(ga, fhat, scales, Yq, Xp, st);
        case 5: return launch_tile<false, 2, 2, 5, 2, 1>(ga, fhat, scales, Yq, Xp, st);
        case 6: return launch_tile<false, 4, 2, 5, 2, 1, 8>(ga, fhat, scales, Yq, Xp, st);
        case 9: return launch_adj_ring<2, 4, 2>(ga, fhat, scales, Yq, Xp, st);
        case 15: return launch_adj_ring<4, 4, 2>(ga, fhat, scales, Yq, Xp, st);
        case 16: return launch_adj_ring<2, 4, 1>(ga, fhat, scales, Yq, Xp, st);
        default: return launch_adj_ring<4, 4, 1>(ga, fhat, scales, Yq, Xp, st);
    }
}

}  // namespace p2o
