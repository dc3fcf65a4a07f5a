// Per-frequency complex matrix-vector products against the stored spectrum.
//
// Section 4 of the paper reduces each matvec, once in Fourier space, to an
// independent Nd x Nm complex matvec per frequency with the block Fhat_w
// (forward) or its conjugate transpose (adjoint), both from one stored copy.
//
// Layout: Fhat is [nfreq][Nd][pitch], complex, real part first, the
// parameter index fastest (pitch >= Nm, a multiple of 32; zero padded).  Both
// directions then stream Fhat once, each lane loading 32 bytes per row as two
// 16-byte halves 1 KB apart (one wavefront load instruction = one contiguous
// kilobyte, whole cache lines; a lane's columns are two runs of V/2):
//  - forward, y_w[i] = sum_j Fhat_w[i, j] x_w[j]: row dot products.  A lane
//    keeps its V entries of x_w in registers and reuses them across every
//    row of the workgroup's slab; partial row sums are reduced across the
//    64-lane wavefront with a multi-value butterfly (about two exchanges per
//    row instead of six), then across the four wavefronts in LDS.  Each
//    column chunk writes its own partial y (no atomics); the inverse FFT
//    that follows adds the partials in a fixed order.
//  - adjoint, x'_w[j] = sum_i conj(Fhat_w[i, j]) y_w[i]: column AXPYs.  A
//    lane owns its V columns and walks the rows; y_w[i] is the same for
//    the whole workgroup (scalar loads).  No cross-lane reduction at all.
// Quantised formats carry one power-of-two multiplier per (frequency,
// 4096-column block).  Forward folds it into x (exact: a power of two);
// adjoint applies it to the finished column sums.
#include "common.hpp"
#include "kernels.hpp"

namespace p2o {

constexpr int kGemvThreads = 256;
constexpr int kMaxFwdRows = 64;

// Reduce N per-lane values across the 64-lane wavefront.  Butterfly steps
// exchange half of the remaining values (offsets 32, 16, ...), so each lane
// ends with one finished sum; plain xor steps finish the rest.  Afterwards
// lanes whose low (6 - log2 N) bits are zero hold value index vidx(lane).
template <typename T, int N>
__device__ __forceinline__ void wave_multi_reduce(T (&v)[N], int lane) {
    static_assert((N & (N - 1)) == 0 && N <= 64, "N must be a power of two <= 64");
    int o = 32;
#pragma unroll
    for (int n = N; n > 1; n >>= 1) {
        const int half = n >> 1;
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const T send = up ? v[i] : v[i + half];
            const T keep = up ? v[i + half] : v[i];
            v[i] = keep + __shfl_xor(send, o);
        }
        o >>= 1;
    }
#pragma unroll
    for (; o >= 1; o >>= 1) v[0] += __shfl_xor(v[0], o);
}

template <int N>
__device__ __forceinline__ int multi_reduce_index(int lane) {
    int idx = 0, o = 32;
#pragma unroll
    for (int n = N; n > 1; n >>= 1) {
        if (lane & o) idx += n >> 1;
        o >>= 1;
    }
    return idx;
}

template <int N>
__device__ __forceinline__ bool multi_reduce_holder(int lane) {
    int steps = 0;
#pragma unroll
    for (int n = N; n > 1; n >>= 1) ++steps;
    return (lane & ((1 << (6 - steps)) - 1)) == 0;
}

// grid: x = column chunk (4 wavefronts x 64 lanes x V columns),
//       y = frequency, z = row slab + nslab * rhs
template <int P, int U>
__global__ __launch_bounds__(kGemvThreads) void k_gemv_fwd(const uint8_t* __restrict__ fhat,
                                                           const float* __restrict__ scales,
                                                           const cplx<typename Fmt<P>::CT>* __restrict__ X,
                                                           cplx<typename Fmt<P>::CT>* __restrict__ Yp,
                                                           GemvArgs ga) {
    using CT = typename Fmt<P>::CT;
    using Z = cplx<CT>;
    constexpr int V = Fmt<P>::V;
    constexpr int B = Fmt<P>::bytes;
    __shared__ CT red[4][kMaxFwdRows][2];

    const int w = blockIdx.y;
    const int b = blockIdx.z / ga.nslab;
    const int slab = blockIdx.z - b * ga.nslab;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // lane columns: col .. col + V/2 - 1 and col + 32 V .. (split 32-byte loads)
    const int col = (blockIdx.x * 4 + wave) * (64 * V) + lane * (V / 2);
    const bool live0 = col < ga.ncols, live1 = col + 32 * V < ga.ncols;

    CT xr[V], xi[V];
    {
        const Z* xp = X + ((long long)w * ga.nrhs + b) * ga.pitch + col;
        CT sc = CT(1);
        if constexpr (Fmt<P>::scaled) sc = live0 ? scales[(long long)w * ga.nblk + col / kScaleBlock] : CT(0);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const bool lv = v < V / 2 ? live0 : live1;
            const Z x = lv ? xp[v < V / 2 ? v : 32 * V + v - V / 2] : Z{CT(0), CT(0)};
            xr[v] = x.x * sc;
            xi[v] = x.y * sc;
        }
    }

    const long long rowb = (long long)ga.pitch * B;
    const uint8_t* Fw = fhat + (long long)w * ga.Nd * rowb + (long long)col * B;
    const int r0 = slab * ga.rows_per_wg;
    const int r1 = min(ga.Nd, r0 + ga.rows_per_wg);

    for (int r = r0; r < r1; r += U) {
        Raw32 raw[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = r + u < r1;
            raw[u] = load32_split(Fw + (long long)(r + u) * rowb, ok && live0, ok && live1);
        }
        CT acc[2 * U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            CT ar[V], ai[V];
            unpack<P>(raw[u], ar, ai);
            CT sr = CT(0), si = CT(0);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                sr += ar[v] * xr[v] - ai[v] * xi[v];
                si += ar[v] * xi[v] + ai[v] * xr[v];
            }
            acc[2 * u] = sr;
            acc[2 * u + 1] = si;
        }
        wave_multi_reduce<CT, 2 * U>(acc, lane);
        if (multi_reduce_holder<2 * U>(lane)) {
            const int vi = multi_reduce_index<2 * U>(lane);
            const int u = vi >> 1;
            if (r + u < r1) red[wave][r - r0 + u][vi & 1] = acc[0];
        }
    }
    __syncthreads();
    const int nrows = r1 - r0;
    Z* out = Yp + (long long)blockIdx.x * ga.part_stride + ((long long)w * ga.nrhs + b) * ga.Nd + r0;
    for (int e = threadIdx.x; e < nrows; e += kGemvThreads) {
        Z y;
        y.x = (red[0][e][0] + red[1][e][0]) + (red[2][e][0] + red[3][e][0]);
        y.y = (red[0][e][1] + red[1][e][1]) + (red[2][e][1] + red[3][e][1]);
        out[e] = y;
    }
}

// grid: x = column group (256 lanes x V columns), y = frequency,
//       z = row slab + nslab * rhs
template <int P, int U>
__global__ __launch_bounds__(kGemvThreads) void k_gemv_adj(const uint8_t* __restrict__ fhat,
                                                           const float* __restrict__ scales,
                                                           const cplx<typename Fmt<P>::CT>* __restrict__ Y,
                                                           cplx<typename Fmt<P>::CT>* __restrict__ Xp,
                                                           GemvArgs ga) {
    using CT = typename Fmt<P>::CT;
    using Z = cplx<CT>;
    constexpr int V = Fmt<P>::V;
    constexpr int B = Fmt<P>::bytes;

    const int w = blockIdx.y;
    const int b = blockIdx.z / ga.nslab;
    const int slab = blockIdx.z - b * ga.nslab;
    // lane columns: col .. col + V/2 - 1 and col + 32 V .. (split 32-byte loads)
    const int col = blockIdx.x * (kGemvThreads * V) + (threadIdx.x >> 6) * (64 * V) + (threadIdx.x & 63) * (V / 2);
    const bool live0 = col < ga.ncols, live1 = col + 32 * V < ga.ncols;
    const int r0 = slab * ga.rows_per_wg;
    const int r1 = min(ga.Nd, r0 + ga.rows_per_wg);

    const long long rowb = (long long)ga.pitch * B;
    const uint8_t* Fw = fhat + (long long)w * ga.Nd * rowb + (long long)col * B;
    const Z* yw = Y + ((long long)w * ga.nrhs + b) * ga.Nd;

    CT accr[V], acci[V];
#pragma unroll
    for (int v = 0; v < V; ++v) { accr[v] = CT(0); acci[v] = CT(0); }

    for (int r = r0; r < r1; r += U) {
        Raw32 raw[U];
        Z y[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = r + u < r1;
            y[u] = ok ? yw[r + u] : Z{CT(0), CT(0)};
            raw[u] = load32_split(Fw + (long long)(r + u) * rowb, ok && live0, ok && live1);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            CT ar[V], ai[V];
            unpack<P>(raw[u], ar, ai);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                accr[v] += ar[v] * y[u].x + ai[v] * y[u].y;
                acci[v] += ar[v] * y[u].y - ai[v] * y[u].x;
            }
        }
    }
    if (live0) {
        CT sc = CT(1);
        if constexpr (Fmt<P>::scaled) sc = scales[(long long)w * ga.nblk + col / kScaleBlock];
        Z* out = Xp + (long long)slab * ga.part_stride + ((long long)w * ga.nrhs + b) * ga.pitch + col;
#pragma unroll
        for (int v = 0; v < V / 2; ++v) out[v] = Z{accr[v] * sc, acci[v] * sc};
        if (live1)
#pragma unroll
            for (int v = V / 2; v < V; ++v) out[32 * V + v - V / 2] = Z{accr[v] * sc, acci[v] * sc};
    }
}

// ---------------------------------------------------------------- host launchers
int gemv_cols_per_lane(int prec) {
    switch (prec) {
        case kFP64: return Fmt<kFP64>::V;
        case kFP32: return Fmt<kFP32>::V;
        case kBF16: return Fmt<kBF16>::V;
        default: return Fmt<kFP16>::V;
    }
}

int gemv_fwd_chunks(int prec, int ncols) {
    const int w = 4 * 64 * gemv_cols_per_lane(prec);
    return (ncols + w - 1) / w;
}

// Rows in flight per lane: 8 x 32 bytes, except FP64 where the wider
// accumulators would cut occupancy.
template <int P> constexpr int fwd_unroll() { return P == kFP64 ? 4 : 8; }

template <int P>
static void fwd_launch(const GemvArgs& ga, const void* fhat, const float* scales, const void* X, void* Yp,
                       hipStream_t st) {
    using Z = cplx<typename Fmt<P>::CT>;
    dim3 grid(gemv_fwd_chunks(P, ga.ncols), ga.nfreq, ga.nslab * ga.nrhs);
    hipLaunchKernelGGL((k_gemv_fwd<P, fwd_unroll<P>()>), grid, dim3(kGemvThreads), 0, st, (const uint8_t*)fhat, scales,
                       (const Z*)X, (Z*)Yp, ga);
}

template <int P>
static void adj_launch(const GemvArgs& ga, const void* fhat, const float* scales, const void* Y, void* Xp,
                       hipStream_t st) {
    using Z = cplx<typename Fmt<P>::CT>;
    const int w = kGemvThreads * Fmt<P>::V;
    dim3 grid((ga.ncols + w - 1) / w, ga.nfreq, ga.nslab * ga.nrhs);
    hipLaunchKernelGGL((k_gemv_adj<P, 8>), grid, dim3(kGemvThreads), 0, st, (const uint8_t*)fhat, scales,
                       (const Z*)Y, (Z*)Xp, ga);
}

hipError_t launch_gemv_fwd(int prec, const GemvArgs& ga, const void* fhat, const float* scales, const void* X,
                           void* Yp, hipStream_t st) {
    if (ga.rows_per_wg > kMaxFwdRows) return hipErrorInvalidValue;
    switch (prec) {
        case kFP64: fwd_launch<kFP64>(ga, fhat, scales, X, Yp, st); break;
        case kFP32: fwd_launch<kFP32>(ga, fhat, scales, X, Yp, st); break;
        case kBF16: fwd_launch<kBF16>(ga, fhat, scales, X, Yp, st); break;
        default: fwd_launch<kFP16>(ga, fhat, scales, X, Yp, st); break;
    }
    return hipGetLastError();
}

hipError_t launch_gemv_adj(int prec, const GemvArgs& ga, const void* fhat, const float* scales, const void* Y,
                           void* Xp, hipStream_t st) {
    switch (prec) {
        case kFP64: adj_launch<kFP64>(ga, fhat, scales, Y, Xp, st); break;
        case kFP32: adj_launch<kFP32>(ga, fhat, scales, Y, Xp, st); break;
        case kBF16: adj_launch<kBF16>(ga, fhat, scales, Y, Xp, st); break;
        default: adj_launch<kFP16>(ga, fhat, scales, Y, Xp, st); break;
    }
    return hipGetLastError();
}

}  // namespace p2o
