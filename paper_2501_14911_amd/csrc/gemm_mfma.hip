// Batched per-frequency products on the matrix cores (many right-hand sides
// per launch): Y_w = Fhat_w X_w and X'_w = Fhat_w^H Y_w for a BF16 spectrum.
//
// With B right-hand sides the per-frequency matvecs of section 4 become one
// complex GEMM per frequency.  Written over the reals with the spectrum in
// its stored interleaved form (re, im, re, im, ... along the parameter
// index), the forward product is a real GEMM of size Nd x 2Nm x 2B: each
// complex right-hand side x contributes the two real columns
// (x_r, -x_i, ...) and (x_i, x_r, ...), whose products with a row are the
// real and imaginary parts of F x.  The adjoint contracts over sensors: with
// K = (sensor, re/im) it is a real GEMM of size Nm x 2Nd x 2B whose two
// columns per right-hand side are (y_r, y_i, ...) and (y_i, -y_r, ...).
//
// Operands.  The spectrum is BF16 and goes to v_mfma_f32_16x16x32_bf16
// as is.  Right-hand sides are FP32 spectra; each value is split into a BF16
// pair hi + lo (hi = RNE(x), lo = RNE(x - hi)), so two MFMAs per tile give
// about 16 significant bits of the right-hand side while accumulating in
// FP32.  The per-(frequency, 4096-column block) power-of-two scale of the
// stored spectrum is folded into x (forward) or the finished columns
// (adjoint); both are exact.
//
// Work.  Every spectrum byte is read once per launch.  Forward workgroups
// own (frequency, 4096-column chunk, 320-row tile, right-hand-side group):
// A fragments stream from HBM straight into registers (each lane loads 32
// contiguous bytes of one row, covering two MFMA K steps), while the right-
// hand sides of the chunk are staged through LDS, double buffered, already
// in fragment order.  The chunk's partial products go to their own slot
// (summed in fixed order by the inverse FFT).  Adjoint workgroups own
// (frequency, 256-column tile): the spectrum tile of 16 sensors x 256
// columns is loaded coalesced and transposed into LDS (rows padded to 20
// words: conflict-free writes, 16-byte fragment reads).  Workgroup ids are
// mapped so that consecutive ids on one XCD share the same frequency (and
// forward column chunk): the right-hand-side spectra they all read stay in
// that XCD's L2.
//
// Any permutation of K inside a lane's 8 values is harmless as long as A
// and B use the same one; both sides below order a lane's values as
// (re, im) pairs of consecutive complex entries.
#include "common.hpp"
#include "kernels.hpp"

namespace p2o {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kGemmThreads = 256;
constexpr int kFwdMB = 5;          // 16-row blocks per wavefront (forward): 320 rows per workgroup
constexpr int kAdjMB = 4;          // 16-column blocks per wavefront (adjoint): 256 columns per workgroup
constexpr int kAdjAW = 20;         // LDS words per transposed column (16 sensors + 4 pad)

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

__device__ __forceinline__ f32x4 mfma(uint4 a, uint4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a), as_bf16x8(b), c, 0, 0, 0);
}

// x = hi + lo with hi, lo BF16 (round to nearest even); returns the raw 16-bit codes.
__device__ __forceinline__ void split_bf16(float x, uint32_t& hi, uint32_t& lo) {
    hi = f32_to_bf16_rne(x);
    lo = f32_to_bf16_rne(x - __uint_as_float(hi << 16));
}

__device__ __forceinline__ int xcd_item(int id, int Q) { return (id & 7) * Q + (id >> 3); }

// Fragment slots in LDS.  A fragment for lane (K group g, column n) is a
// 16-byte chunk; the chunk's bank quad is its slot mod 16.  Rotating the slot
// by the K group (and K half) spreads the staging writes of one wavefront
// over all 64 banks, while each 16-lane phase of the fragment reads still
// touches 16 distinct quads.
__device__ __forceinline__ int fwd_slot(int g, int n, int h) { return g * 16 + ((n + 4 * g + h) & 15); }
__device__ __forceinline__ int adj_slot(int g, int n) { return g * 16 + ((n + (g & 1) + 8 * (g >> 1)) & 15); }

// ---------------------------------------------------------------- forward
template <int NB>
__global__ __launch_bounds__(kGemmThreads) void k_gemm_fwd(const uint8_t* __restrict__ fhat,
                                                           const float* __restrict__ scales,
                                                           const float2* __restrict__ X,
                                                           float2* __restrict__ Yp, GemmArgs ga) {
    constexpr int MB = kFwdMB;
    constexpr int RB = 8 * NB;                 // right-hand sides per group (16 real columns per block)
    constexpr int ROWS = 4 * MB * 16;
    __shared__ uint4 bs[2][NB][2][2][64];      // [buffer][n block][K half][hi/lo][lane]

    const int q = xcd_item(blockIdx.x, ga.Q);
    if (q >= ga.items) return;
    int t = q;
    const int mt = t % ga.n_mt; t /= ga.n_mt;
    const int bg = t % ga.n_bg; t /= ga.n_bg;
    const int kc = t % ga.n_kc; t /= ga.n_kc;
    const int w = t;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lg = lane >> 4;
    const int b0 = bg * RB;
    const int jbeg = kc * ga.kchunk;
    const int jend = min(ga.pitch, jbeg + ga.kchunk);
    const int nsteps = (jend - jbeg + 31) >> 5;
    const float sc = scales[(long long)w * ga.nblk + jbeg / kScaleBlock];

    const int rowbase = mt * ROWS + wave * MB * 16;
    const uint8_t* arow[MB];
    bool rok[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const int row = rowbase + mb * 16 + lr;
        rok[mb] = row < ga.Nd;
        arow[mb] = fhat + (((long long)w * ga.Nd + (rok[mb] ? row : 0)) * ga.pitch + jbeg + 8 * lg) * 4;
    }
    auto load_a = [&](Raw32 (&a)[MB], int s) {
        const int j = jbeg + 32 * s + 8 * lg;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            if (rok[mb] && j < jend) a[mb] = load32(arow[mb] + (long long)s * 128);
            else a[mb] = Raw32{make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0)};
        }
    };

    f32x4 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

    // right-hand-side values a thread stages per step (32 columns x RB)
    constexpr int XPT = (32 * RB + kGemmThreads - 1) / kGemmThreads;
    const float2* Xw = X + (long long)w * ga.nrhs * ga.pitch;
    auto load_x = [&](float2 (&xv)[XPT], int s) {
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int e = tid + u * kGemmThreads;
            const int c = e & 31, bl = e >> 5;
            const int b = b0 + bl, j = jbeg + 32 * s + c;
            xv[u] = (e < 32 * RB && b < ga.nrhs && j < jend) ? Xw[(long long)b * ga.pitch + j] : make_float2(0.f, 0.f);
        }
    };
    // BF16 hi/lo fragments in [n block][K half][hi/lo][lane] order
    auto stage_x = [&](const float2 (&xv)[XPT], int buf) {
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int e = tid + u * kGemmThreads;
            if (e >= 32 * RB) break;
            const int c = e & 31, bl = e >> 5;
            uint32_t rh, rl, ih, il;
            split_bf16(xv[u].x * sc, rh, rl);
            split_bf16(xv[u].y * sc, ih, il);
            const int g = c >> 3, h = (c >> 2) & 1, cc = c & 3;
            const int nre = 2 * bl, nim = 2 * bl + 1;
            // real-part column: (x_r, -x_i); imaginary-part column: (x_i, x_r)
            const int sre = fwd_slot(g, nre & 15, h), sim = fwd_slot(g, nim & 15, h);
            reinterpret_cast<uint32_t*>(&bs[buf][nre >> 4][h][0][sre])[cc] = rh | ((ih ^ 0x8000u) << 16);
            reinterpret_cast<uint32_t*>(&bs[buf][nre >> 4][h][1][sre])[cc] = rl | ((il ^ 0x8000u) << 16);
            reinterpret_cast<uint32_t*>(&bs[buf][nim >> 4][h][0][sim])[cc] = ih | (rh << 16);
            reinterpret_cast<uint32_t*>(&bs[buf][nim >> 4][h][1][sim])[cc] = il | (rl << 16);
        }
    };
    auto compute = [&](const Raw32 (&a)[MB], int buf) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int s0 = fwd_slot(lg, lr, 0), s1 = fwd_slot(lg, lr, 1);
            const uint4 f0h = bs[buf][nb][0][0][s0], f0l = bs[buf][nb][0][1][s0];
            const uint4 f1h = bs[buf][nb][1][0][s1], f1l = bs[buf][nb][1][1][s1];
            // consecutive MFMAs use different accumulators (no dependent issue)
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb][nb] = mfma(a[mb].a, f0h, acc[mb][nb]);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb][nb] = mfma(a[mb].a, f0l, acc[mb][nb]);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb][nb] = mfma(a[mb].b, f1h, acc[mb][nb]);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb][nb] = mfma(a[mb].b, f1l, acc[mb][nb]);
        }
    };

    // two register sets: loads for step s + 2 are in flight while step s computes
    Raw32 a0[MB], a1[MB];
    float2 x0[XPT], x1[XPT];
    load_a(a0, 0);
    load_x(x0, 0);
    if (nsteps > 1) { load_a(a1, 1); load_x(x1, 1); }
    for (int s = 0; s < nsteps; s += 2) {
        stage_x(x0, 0);
        if (s + 2 < nsteps) load_x(x0, s + 2);
        __syncthreads();
        compute(a0, 0);
        if (s + 2 < nsteps) load_a(a0, s + 2);
        if (s + 1 < nsteps) {
            stage_x(x1, 1);
            if (s + 3 < nsteps) load_x(x1, s + 3);
            __syncthreads();
            compute(a1, 1);
            if (s + 3 < nsteps) load_a(a1, s + 3);
        }
    }

    // partial sums of this column chunk: Yp[kc][w][b][row], row-block lanes hold rows 4 lg + r
    float* out = reinterpret_cast<float*>(Yp + (long long)kc * ga.part_stride + (long long)w * ga.nrhs * ga.Nd);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int ncol = nb * 16 + lr;
        const int b = b0 + (ncol >> 1), comp = ncol & 1;
        if (b >= ga.nrhs) continue;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rowbase + mb * 16 + 4 * lg + r;
                if (row < ga.Nd) out[2 * ((long long)b * ga.Nd + row) + comp] = acc[mb][nb][r];
            }
        }
    }
}

// ---------------------------------------------------------------- adjoint
template <int NB>
__global__ __launch_bounds__(kGemmThreads) void k_gemm_adj(const uint8_t* __restrict__ fhat,
                                                           const float* __restrict__ scales,
                                                           const float2* __restrict__ Y,
                                                           float2* __restrict__ Xp, GemmArgs ga) {
    constexpr int MB = kAdjMB;
    constexpr int RB = 8 * NB;
    constexpr int COLS = 4 * MB * 16;
    __shared__ uint32_t as[2][COLS * kAdjAW];  // [buffer][column][sensor + pad]
    __shared__ uint4 bs[2][NB][2][64];         // [buffer][n block][hi/lo][lane]

    const int q = xcd_item(blockIdx.x, ga.Q);
    if (q >= ga.items) return;
    int t = q;
    const int jt = t % ga.n_mt; t /= ga.n_mt;
    const int bg = t % ga.n_bg; t /= ga.n_bg;
    const int w = t;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lg = lane >> 4;
    const int b0 = bg * RB;
    const int j0 = jt * COLS;
    const int nsteps = (ga.Nd + 15) >> 4;
    const uint8_t* Fw = fhat + (long long)w * ga.Nd * ga.pitch * 4;
    const float2* Yw = Y + (long long)w * ga.nrhs * ga.Nd;

    f32x4 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};

    // per-thread share of one step: spectrum tile (16 x COLS/4 chunks of 16 B)
    // and right-hand sides (16 x RB values)
    constexpr int APT = (16 * (COLS / 4) + kGemmThreads - 1) / kGemmThreads;
    constexpr int BPT = (16 * RB + kGemmThreads - 1) / kGemmThreads;
    auto load_ab = [&](uint4 (&av)[APT], float2 (&bv)[BPT], int s) {
        const int i0 = 16 * s;
#pragma unroll
        for (int u = 0; u < APT; ++u) {
            const int e = tid + u * kGemmThreads;
            const int r = e & 15, ch = e >> 4;
            const int i = i0 + r, j = j0 + 4 * ch;
            av[u] = make_uint4(0, 0, 0, 0);
            if (e < 16 * (COLS / 4) && i < ga.Nd && j < ga.pitch) {
                const u32x4 raw = __builtin_nontemporal_load(
                    reinterpret_cast<const u32x4*>(Fw + ((long long)i * ga.pitch + j) * 4));
                av[u] = make_uint4(raw.x, raw.y, raw.z, raw.w);
            }
        }
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            const int e = tid + u * kGemmThreads;
            const int r = e & 15, bl = e >> 4;
            const int b = b0 + bl, i = i0 + r;
            bv[u] = (e < 16 * RB && b < ga.nrhs && i < ga.Nd) ? Yw[(long long)b * ga.Nd + i] : make_float2(0.f, 0.f);
        }
    };
    auto stage_ab = [&](const uint4 (&av)[APT], const float2 (&bv)[BPT], int buf) {
#pragma unroll
        for (int u = 0; u < APT; ++u) {
            const int e = tid + u * kGemmThreads;
            if (e >= 16 * (COLS / 4)) break;
            const int r = e & 15, ch = e >> 4;
            uint32_t* dst = &as[buf][(4 * ch) * kAdjAW + r];     // transposed to [column][sensor]
            dst[0] = av[u].x;
            dst[kAdjAW] = av[u].y;
            dst[2 * kAdjAW] = av[u].z;
            dst[3 * kAdjAW] = av[u].w;
        }
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            const int e = tid + u * kGemmThreads;
            if (e >= 16 * RB) break;
            const int r = e & 15, bl = e >> 4;
            uint32_t rh, rl, ih, il;
            split_bf16(bv[u].x, rh, rl);
            split_bf16(bv[u].y, ih, il);
            const int g = r >> 2, rho = r & 3;
            const int nre = 2 * bl, nim = 2 * bl + 1;
            // real-part column: (y_r, y_i); imaginary-part column: (y_i, -y_r)
            const int sre = adj_slot(g, nre & 15), sim = adj_slot(g, nim & 15);
            reinterpret_cast<uint32_t*>(&bs[buf][nre >> 4][0][sre])[rho] = rh | (ih << 16);
            reinterpret_cast<uint32_t*>(&bs[buf][nre >> 4][1][sre])[rho] = rl | (il << 16);
            reinterpret_cast<uint32_t*>(&bs[buf][nim >> 4][0][sim])[rho] = ih | ((rh ^ 0x8000u) << 16);
            reinterpret_cast<uint32_t*>(&bs[buf][nim >> 4][1][sim])[rho] = il | ((rl ^ 0x8000u) << 16);
        }
    };
    auto compute = [&](int buf) {
        uint4 afr[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int col = wave * MB * 16 + mb * 16 + lr;
            afr[mb] = *reinterpret_cast<const uint4*>(&as[buf][col * kAdjAW + 4 * lg]);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int sl = adj_slot(lg, lr);
            const uint4 fh = bs[buf][nb][0][sl], fl = bs[buf][nb][1][sl];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb][nb] = mfma(afr[mb], fh, acc[mb][nb]);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) acc[mb][nb] = mfma(afr[mb], fl, acc[mb][nb]);
        }
    };

    // two register sets: loads for step s + 2 are in flight while step s computes
    uint4 av0[APT], av1[APT];
    float2 bv0[BPT], bv1[BPT];
    load_ab(av0, bv0, 0);
    if (nsteps > 1) load_ab(av1, bv1, 1);
    for (int s = 0; s < nsteps; s += 2) {
        stage_ab(av0, bv0, 0);
        if (s + 2 < nsteps) load_ab(av0, bv0, s + 2);
        __syncthreads();
        compute(0);
        if (s + 1 < nsteps) {
            stage_ab(av1, bv1, 1);
            if (s + 3 < nsteps) load_ab(av1, bv1, s + 3);
            __syncthreads();
            compute(1);
        }
    }

    const float sc = scales[(long long)w * ga.nblk + j0 / kScaleBlock];
    float* out = reinterpret_cast<float*>(Xp + (long long)w * ga.nrhs * ga.pitch);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        const int ncol = nb * 16 + lr;
        const int b = b0 + (ncol >> 1), comp = ncol & 1;
        if (b >= ga.nrhs) continue;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = j0 + wave * MB * 16 + mb * 16 + 4 * lg + r;
                if (j < ga.pitch) out[2 * ((long long)b * ga.pitch + j) + comp] = acc[mb][nb][r] * sc;
            }
        }
    }
}

// ---------------------------------------------------------------- host launchers
static int gemm_nb(int nrhs) { return nrhs > 32 ? 8 : nrhs > 16 ? 4 : nrhs > 8 ? 2 : 1; }

int gemm_fwd_kchunks(int pitch) { return (pitch + kScaleBlock - 1) / kScaleBlock; }

hipError_t launch_gemm_fwd(const GemmArgs& in, const void* fhat, const float* scales, const void* X, void* Yp,
                           hipStream_t st) {
    GemmArgs ga = in;
    const int NB = gemm_nb(ga.nrhs);
    ga.kchunk = kScaleBlock;
    ga.n_kc = gemm_fwd_kchunks(ga.pitch);
    ga.n_mt = (ga.Nd + 4 * kFwdMB * 16 - 1) / (4 * kFwdMB * 16);
    ga.n_bg = (ga.nrhs + 8 * NB - 1) / (8 * NB);
    ga.items = ga.nfreq * ga.n_kc * ga.n_bg * ga.n_mt;
    ga.Q = (ga.items + 7) / 8;
    dim3 grid(8 * ga.Q);
    const uint8_t* F = (const uint8_t*)fhat;
    const float2* x = (const float2*)X;
    float2* y = (float2*)Yp;
    switch (NB) {
        case 8: hipLaunchKernelGGL((k_gemm_fwd<8>), grid, dim3(kGemmThreads), 0, st, F, scales, x, y, ga); break;
        case 4: hipLaunchKernelGGL((k_gemm_fwd<4>), grid, dim3(kGemmThreads), 0, st, F, scales, x, y, ga); break;
        case 2: hipLaunchKernelGGL((k_gemm_fwd<2>), grid, dim3(kGemmThreads), 0, st, F, scales, x, y, ga); break;
        default: hipLaunchKernelGGL((k_gemm_fwd<1>), grid, dim3(kGemmThreads), 0, st, F, scales, x, y, ga); break;
    }
    return hipGetLastError();
}

hipError_t launch_gemm_adj(const GemmArgs& in, const void* fhat, const float* scales, const void* Y, void* Xp,
                           hipStream_t st) {
    GemmArgs ga = in;
    const int NB = gemm_nb(ga.nrhs);
    ga.n_mt = (ga.pitch + 4 * kAdjMB * 16 - 1) / (4 * kAdjMB * 16);
    ga.n_kc = 1;
    ga.n_bg = (ga.nrhs + 8 * NB - 1) / (8 * NB);
    ga.items = ga.nfreq * ga.n_bg * ga.n_mt;
    ga.Q = (ga.items + 7) / 8;
    dim3 grid(8 * ga.Q);
    const uint8_t* F = (const uint8_t*)fhat;
    const float2* y = (const float2*)Y;
    float2* x = (float2*)Xp;
    switch (NB) {
        case 8: hipLaunchKernelGGL((k_gemm_adj<8>), grid, dim3(kGemmThreads), 0, st, F, scales, y, x, ga); break;
        case 4: hipLaunchKernelGGL((k_gemm_adj<4>), grid, dim3(kGemmThreads), 0, st, F, scales, y, x, ga); break;
        case 2: hipLaunchKernelGGL((k_gemm_adj<2>), grid, dim3(kGemmThreads), 0, st, F, scales, y, x, ga); break;
        default: hipLaunchKernelGGL((k_gemm_adj<1>), grid, dim3(kGemmThreads), 0, st, F, scales, y, x, ga); break;
    }
    return hipGetLastError();
}

}  // namespace p2o
