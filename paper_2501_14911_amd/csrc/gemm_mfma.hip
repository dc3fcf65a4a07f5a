// Batched per-frequency products on the matrix cores (many right-hand sides
// per launch): Y_w = Fhat_w X_w and X'_w = Fhat_w^H Y_w for a BF16 spectrum.
//
// With B right-hand sides the per-frequency matvecs of section 4 become one
// complex GEMM per frequency, done with v_mfma_f32_32x32x16_bf16 (on gfx950
// the 32x32 shape sustains about 1.5x the rate of the 16x16x32 one, and
// does so with one wavefront per SIMD).  K runs over (index, re/im) pairs in
// their stored interleaved order, so a complex product is two real ones
// against forms of the spectrum fragment, each 32-bit word (re, im) being
// rewritten by one or two VALU operations:
//   forward  y_r = (a_r, -a_i) . (x_r, x_i)   y_i = (a_i, a_r) . (x_r, x_i)
//   adjoint  x_r = (a_r,  a_i) . (y_r, y_i)   x_i = (-a_i, a_r) . (y_r, y_i)
// (the adjoint takes conj(F)^T).  Right-hand sides arrive as quad BF16 hi/lo
// storage (written by the FFT that produced them); hi and lo each go through
// the matrix cores, giving about 16 significant bits of x with FP32
// accumulation.  The per-(frequency, 4096-column block) power-of-two scale of
// the stored spectrum multiplies finished outputs (exact).
//
// Work.  A workgroup is 4 wavefronts, each owning 3 (or 5) blocks of 32
// output rows (forward: sensors; adjoint: parameter columns) for 64 (or 32)
// right-hand sides; the 4 share the right-hand sides of each K step through
// LDS.  Spectrum fragments are loaded by each lane straight into registers
// (no LDS), one pipeline step (4 K substeps of 8 complex entries) ahead of
// the matrix cores; there is no cross-wave reuse of the spectrum to exploit,
// and registers hold more bytes in flight than LDS could.  Forward lanes
// load 16 bytes of a row per substep, so each row is read in 128-byte runs
// per step; adjoint lanes gather 4 sensors of one column as 4-byte words
// from 4 rows, each wavefront load covering 128 contiguous bytes of two rows.
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

constexpr int kGemmThreads = 256;
constexpr int kU = 4;              // K substeps (8 complex entries, 16 real K) per pipeline step

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
__device__ __forceinline__ uint4 f_jrot(uint4 a) {                       // (-im, re)
    return make_uint4(w_swap(a.x) ^ 0x8000u, w_swap(a.y) ^ 0x8000u, w_swap(a.z) ^ 0x8000u, w_swap(a.w) ^ 0x8000u);
}

__device__ __forceinline__ int xcd_item(int id, int Q) { return (id & 7) * Q + (id >> 3); }

// Workgroup barrier that waits for this wavefront's LDS operations but not
// for its loads in flight (__syncthreads would also drain the spectrum
// prefetch).  The empty asm statements keep the compiler from moving memory
// accesses across it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);      // lgkmcnt(0); vmcnt, expcnt not waited on
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Right-hand sides of one pipeline step: 8 groups of 4 consecutive K entries
// (columns or sensors) for 32 NB right-hand sides, loaded cooperatively and
// stored in LDS as B fragments [substep][n block][hi/lo][lane] (16 bytes per
// lane: lane n + 32 g holds the 4 entries of group 2 substep + g of
// right-hand side n).  Groups at or past glim are zero; right-hand sides past
// the last valid one repeat it (their outputs are never stored).
template <int NB>
struct RhsStage {
    static constexpr int PAIRS = 32 * NB * 2 * kU;
    static constexpr int PT = PAIRS / kGemmThreads;
    static_assert(PT * kGemmThreads == PAIRS, "pairs per thread");
    uint4 h[PT], l[PT];
    uint32_t m[PT];           // all ones for groups below glim, else zero (applied when stored)

    __device__ __forceinline__ void load(const uint8_t* rows, long long ld_bytes, int nb_valid, int g0, int glim,
                                         int tid) {
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const int p = tid + i * kGemmThreads;
            const int g = p & (2 * kU - 1), bl = min(p >> 3, nb_valid - 1);
            const int gi = g0 + g;
            const bool ok = gi < glim;
            const uint4* src = reinterpret_cast<const uint4*>(rows + bl * ld_bytes + (long long)(ok ? gi : 0) * 32);
            h[i] = src[0];
            l[i] = src[1];
            m[i] = ok ? 0xffffffffu : 0u;
        }
    }
    __device__ __forceinline__ void store(uint4 (*bf)[NB][2][64], int tid) const {
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const int p = tid + i * kGemmThreads;
            const int g = p & (2 * kU - 1), bl = p >> 3;
            const int lane = (bl & 31) + 32 * (g & 1);
            const uint32_t k = m[i];
            bf[g >> 1][bl >> 5][0][lane] = make_uint4(h[i].x & k, h[i].y & k, h[i].z & k, h[i].w & k);
            bf[g >> 1][bl >> 5][1][lane] = make_uint4(l[i].x & k, l[i].y & k, l[i].z & k, l[i].w & k);
        }
    }
};

// ---------------------------------------------------------------- forward
// Yp[kc][w][b][row] = scale * sum over the chunk's columns j of F[w][row][j] x_b[w][j]
template <int MB, int NB>
__global__ __launch_bounds__(kGemmThreads) void k_gemm_fwd(const uint8_t* fhat,
                                                           const float* __restrict__ scales,
                                                           const uint8_t* Xq,
                                                           float2* __restrict__ Yp, GemmArgs ga) {
    __shared__ __align__(16) uint4 bfr[2][kU][NB][2][64];

    const int q = xcd_item(blockIdx.x, ga.Q);
    if (q >= ga.items) return;
    int t = q;
    const int mt = t % ga.n_mt; t /= ga.n_mt;
    const int bg = t % ga.n_bg; t /= ga.n_bg;
    const int kc = t % ga.n_kc; t /= ga.n_kc;
    const int w = t;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = lane & 31, kg = lane >> 5;
    const int b0 = bg * 32 * NB;
    const int nb_valid = min(32 * NB, ga.nrhs - b0);
    const int jbeg = kc * ga.kchunk;
    const int jend = min(ga.pitch, jbeg + ga.kchunk);
    const int nst = (jend - jbeg + 8 * kU - 1) / (8 * kU);
    const int row0 = (mt * 4 + wave) * 32 * MB;

    // lane (r, kg) of m block mb reads row row0 + 32 mb + r, columns 4 kg ..
    // 4 kg + 3 of each substep.  Rows past Nd repeat the last one (their
    // outputs are not stored); the wavefronts of a workgroup move in step, so
    // computing them costs no time.
    const uint8_t* arow[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const int row = min(row0 + 32 * mb + r, ga.Nd - 1);
        arow[mb] = fhat + (((long long)w * ga.Nd + row) * ga.pitch + 4 * kg) * 4;
    }
    auto load_a = [&](uint4 (&a)[MB][kU], int st) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            int j = jbeg + st * 8 * kU + 8 * u;
            if (j >= jend) j = jbeg;                 // past the chunk: B is zero there
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) a[mb][u] = *reinterpret_cast<const uint4*>(arow[mb] + (long long)j * 4);
        }
    };
    const uint8_t* xrows = Xq + ((long long)w * ga.nrhs + b0) * ga.ldb * 8;
    const long long ldb_bytes = (long long)ga.ldb * 8;
    auto load_b = [&](RhsStage<NB>& rs, int st) {
        rs.load(xrows, ldb_bytes, nb_valid, (jbeg + st * 8 * kU) / 4, jend / 4, tid);
    };

    f32x16 accr[MB][NB], acci[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) accr[mb][nb] = acci[mb][nb] = f32x16{};

    auto compute = [&](const uint4 (&a)[MB][kU], int buf) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            __builtin_amdgcn_sched_barrier(0);
            uint4 bh[NB], bl[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                bh[nb] = bfr[buf][u][nb][0][lane];
                bl[nb] = bfr[buf][u][nb][1][lane];
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const uint4 a1 = f_conj(a[mb][u]), a2 = f_swap(a[mb][u]);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    accr[mb][nb] = mfma32(a1, bh[nb], accr[mb][nb]);
                    acci[mb][nb] = mfma32(a2, bh[nb], acci[mb][nb]);
                    accr[mb][nb] = mfma32(a1, bl[nb], accr[mb][nb]);
                    acci[mb][nb] = mfma32(a2, bl[nb], acci[mb][nb]);
                }
            }
        }
    };

// Step st of the pipeline (both directions): stage B(st+1), loaded one step
    // earlier, into the LDS buffer step st-1 read; load B(st+2); prefetch
    // A(st+2) into the buffer step st-1 used; compute step st; barrier.
    // Loads retire in order and B(st+1) was issued before A(st+1), so waiting
    // for it leaves A(st+1) and A(st+2) in flight: every A prefetch has two
    // compute phases to arrive.  Prefetches past the last step repeat it (A)
    // or read zeros (B) and are never used; the step has no branches.
    uint4 a0[MB][kU], a1[MB][kU], a2[MB][kU];
    RhsStage<NB> rs;
    auto step = [&](const uint4 (&cur)[MB][kU], uint4 (&pre)[MB][kU], int st) {
        rs.store(bfr[(st + 1) & 1], tid);
        load_b(rs, st + 2);
        load_a(pre, min(st + 2, nst - 1));
        compute(cur, st & 1);
        lds_barrier();
    };
    load_b(rs, 0);
    load_a(a0, 0);
    rs.store(bfr[0], tid);
    load_b(rs, 1);
    load_a(a1, min(1, nst - 1));
    lds_barrier();
    int st = 0;
    for (; st + 3 <= nst; st += 3) {
        step(a0, a2, st);
        step(a1, a0, st + 1);
        step(a2, a1, st + 2);
    }
    if (st < nst) step(a0, a2, st);
    if (st + 1 < nst) step(a1, a0, st + 1);

    // output tile (32 rows x 32 right-hand sides): lane (n, h) holds rows
    // 8 (v / 4) + 4 h + v % 4 of column n in element v
    const float sc = scales[(long long)w * ga.nblk + jbeg / kScaleBlock];
    float2* out = Yp + (long long)kc * ga.part_stride + (long long)w * ga.nrhs * ga.Nd;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int b = b0 + 32 * nb + r;
        if (b >= ga.nrhs) continue;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = row0 + 32 * mb + 8 * (v >> 2) + 4 * kg + (v & 3);
                if (row < ga.Nd)
                    out[(long long)b * ga.Nd + row] = make_float2(accr[mb][nb][v] * sc, acci[mb][nb][v] * sc);
            }
        }
    }
}

// ---------------------------------------------------------------- adjoint
// Xp[w][b][j] = scale_j * sum over sensors i of conj(F[w][i][j]) y_b[w][i]
template <int MB, int NB>
__global__ __launch_bounds__(kGemmThreads) void k_gemm_adj(const uint8_t* fhat,
                                                           const float* __restrict__ scales,
                                                           const uint8_t* Yq,
                                                           float2* __restrict__ Xp, GemmArgs ga) {
    __shared__ __align__(16) uint4 bfr[2][kU][NB][2][64];

    const int q = xcd_item(blockIdx.x, ga.Q);
    if (q >= ga.items) return;
    int t = q;
    const int jt = t % ga.n_mt; t /= ga.n_mt;
    const int bg = t % ga.n_bg; t /= ga.n_bg;
    const int w = t;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int c = lane & 31, kg = lane >> 5;
    const int b0 = bg * 32 * NB;
    const int nb_valid = min(32 * NB, ga.nrhs - b0);
    const int col0 = (jt * 4 + wave) * 32 * MB;
    const int nst = (ga.ldb + 8 * kU - 1) / (8 * kU);

    // lane (c, kg) of m block mb reads column col0 + 32 mb + c, sensors
    // 4 kg .. 4 kg + 3 of each substep (rows past Nd repeat the last one:
    // their B entries are zero; columns past the pitch repeat the last one
    // and are not stored)
    const uint32_t* Fw = reinterpret_cast<const uint32_t*>(fhat) + (long long)w * ga.Nd * ga.pitch;
    int jcol[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) jcol[mb] = min(col0 + 32 * mb + c, ga.pitch - 1);
    auto load_a = [&](uint4 (&a)[MB][kU], int st) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int i0 = st * 8 * kU + 8 * u + 4 * kg;
            const uint32_t* r0 = Fw + (long long)min(i0, ga.Nd - 1) * ga.pitch;
            const uint32_t* r1 = Fw + (long long)min(i0 + 1, ga.Nd - 1) * ga.pitch;
            const uint32_t* r2 = Fw + (long long)min(i0 + 2, ga.Nd - 1) * ga.pitch;
            const uint32_t* r3 = Fw + (long long)min(i0 + 3, ga.Nd - 1) * ga.pitch;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) a[mb][u] = make_uint4(r0[jcol[mb]], r1[jcol[mb]], r2[jcol[mb]], r3[jcol[mb]]);
        }
    };
    const uint8_t* yrows = Yq + ((long long)w * ga.nrhs + b0) * ga.ldb * 8;
    const long long ldb_bytes = (long long)ga.ldb * 8;
    auto load_b = [&](RhsStage<NB>& rs, int st) {
        rs.load(yrows, ldb_bytes, nb_valid, st * 2 * kU, ga.ldb / 4, tid);
    };

    f32x16 accr[MB][NB], acci[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) accr[mb][nb] = acci[mb][nb] = f32x16{};

    auto compute = [&](const uint4 (&a)[MB][kU], int buf) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            __builtin_amdgcn_sched_barrier(0);
            uint4 bh[NB], bl[NB];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                bh[nb] = bfr[buf][u][nb][0][lane];
                bl[nb] = bfr[buf][u][nb][1][lane];
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const uint4 a1 = a[mb][u], a2 = f_jrot(a[mb][u]);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    accr[mb][nb] = mfma32(a1, bh[nb], accr[mb][nb]);
                    acci[mb][nb] = mfma32(a2, bh[nb], acci[mb][nb]);
                    accr[mb][nb] = mfma32(a1, bl[nb], accr[mb][nb]);
                    acci[mb][nb] = mfma32(a2, bl[nb], acci[mb][nb]);
                }
            }
        }
    };

// Step st of the pipeline (both directions): stage B(st+1), loaded one step
    // earlier, into the LDS buffer step st-1 read; load B(st+2); prefetch
    // A(st+2) into the buffer step st-1 used; compute step st; barrier.
    // Loads retire in order and B(st+1) was issued before A(st+1), so waiting
    // for it leaves A(st+1) and A(st+2) in flight: every A prefetch has two
    // compute phases to arrive.  Prefetches past the last step repeat it (A)
    // or read zeros (B) and are never used; the step has no branches.
    uint4 a0[MB][kU], a1[MB][kU], a2[MB][kU];
    RhsStage<NB> rs;
    auto step = [&](const uint4 (&cur)[MB][kU], uint4 (&pre)[MB][kU], int st) {
        rs.store(bfr[(st + 1) & 1], tid);
        load_b(rs, st + 2);
        load_a(pre, min(st + 2, nst - 1));
        compute(cur, st & 1);
        lds_barrier();
    };
    load_b(rs, 0);
    load_a(a0, 0);
    rs.store(bfr[0], tid);
    load_b(rs, 1);
    load_a(a1, min(1, nst - 1));
    lds_barrier();
    int st = 0;
    for (; st + 3 <= nst; st += 3) {
        step(a0, a2, st);
        step(a1, a0, st + 1);
        step(a2, a1, st + 2);
    }
    if (st < nst) step(a0, a2, st);
    if (st + 1 < nst) step(a1, a0, st + 1);

    // output tile (32 columns x 32 right-hand sides); an m block lies in one
    // 4096-column scale block
    float2* out = Xp + (long long)w * ga.nrhs * ga.pitch;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const int jb = col0 + 32 * mb;
        if (jb >= ga.pitch) continue;
        const float sc = scales[(long long)w * ga.nblk + jb / kScaleBlock];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int b = b0 + 32 * nb + c;
            if (b >= ga.nrhs) continue;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int j = jb + 8 * (v >> 2) + 4 * kg + (v & 3);
                if (j < ga.pitch)
                    out[(long long)b * ga.pitch + j] = make_float2(accr[mb][nb][v] * sc, acci[mb][nb][v] * sc);
            }
        }
    }
}

// ---------------------------------------------------------------- host launchers
int gemm_fwd_kchunks(int pitch) { return (pitch + kScaleBlock - 1) / kScaleBlock; }

int gemm_data_pitch(int Nd) { return (Nd + 7) / 8 * 8; }

hipError_t launch_gemm_fwd(const GemmArgs& in, const void* fhat, const float* scales, const void* Xq, void* Yp,
                           hipStream_t st) {
    GemmArgs ga = in;
    const bool wide = ga.nrhs > 32;
    const int MB = wide ? 3 : 5, NB = wide ? 2 : 1;
    ga.ldb = ga.pitch;
    ga.kchunk = kScaleBlock;
    ga.n_kc = gemm_fwd_kchunks(ga.pitch);
    ga.n_mt = (ga.Nd + 4 * 32 * MB - 1) / (4 * 32 * MB);
    ga.n_bg = (ga.nrhs + 32 * NB - 1) / (32 * NB);
    ga.items = ga.nfreq * ga.n_kc * ga.n_bg * ga.n_mt;
    ga.Q = (ga.items + 7) / 8;
    dim3 grid(8 * ga.Q);
    const uint8_t* F = (const uint8_t*)fhat;
    const uint8_t* x = (const uint8_t*)Xq;
    float2* y = (float2*)Yp;
    if (wide) hipLaunchKernelGGL((k_gemm_fwd<3, 2>), grid, dim3(kGemmThreads), 0, st, F, scales, x, y, ga);
    else hipLaunchKernelGGL((k_gemm_fwd<5, 1>), grid, dim3(kGemmThreads), 0, st, F, scales, x, y, ga);
    return hipGetLastError();
}

hipError_t launch_gemm_adj(const GemmArgs& in, const void* fhat, const float* scales, const void* Yq, void* Xp,
                           hipStream_t st) {
    GemmArgs ga = in;
    const bool wide = ga.nrhs > 32;
    const int MB = wide ? 3 : 5, NB = wide ? 2 : 1;
    ga.ldb = gemm_data_pitch(ga.Nd);
    ga.n_mt = (ga.pitch + 4 * 32 * MB - 1) / (4 * 32 * MB);
    ga.n_kc = 1;
    ga.n_bg = (ga.nrhs + 32 * NB - 1) / (32 * NB);
    ga.items = ga.nfreq * ga.n_bg * ga.n_mt;
    ga.Q = (ga.items + 7) / 8;
    dim3 grid(8 * ga.Q);
    const uint8_t* F = (const uint8_t*)fhat;
    const uint8_t* y = (const uint8_t*)Yq;
    float2* x = (float2*)Xp;
    if (wide) hipLaunchKernelGGL((k_gemm_adj<3, 2>), grid, dim3(kGemmThreads), 0, st, F, scales, y, x, ga);
    else hipLaunchKernelGGL((k_gemm_adj<5, 1>), grid, dim3(kGemmThreads), 0, st, F, scales, y, x, ga);
    return hipGetLastError();
}

}  // namespace p2o
