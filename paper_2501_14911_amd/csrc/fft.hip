// Batched real FFTs along time for the block-Toeplitz matvec.
//
// Section 4 of the paper embeds the block lower-triangular Toeplitz matrix
// in a block circulant of length L and diagonalises it with the DFT: every
// time series (one per parameter or sensor) is zero-padded to L, transformed,
// multiplied per frequency, transformed back and truncated to Nt steps.
//
// Design for gfx950.  Series are the contiguous dimension of time-major
// arrays, so a workgroup takes a tile of TW adjacent series and all time
// steps: every global access is a run of TW consecutive elements.  The tile
// lives in LDS as [bin][series].  A real series x of even length L is
// transformed as one complex series z[n] = x[2n] + i x[2n+1] of length
// M = L/2 (half the work and LDS), followed by the usual split into the
// spectra of the even and odd samples.  The complex transform is a
// Stockham autosort FFT (Govindaraju et al., "High performance discrete
// Fourier transforms on graphics processors", SC'08) with radices
// 8, 4, 2, 3, 5, 7, run in place: each pass stages its butterflies' inputs
// in registers, synchronises, then writes.  Twiddles come from a table
// e^{-2 pi i n / L} generated once per plan in FP64 with sincospi.
//
// Zero padding (inputs past Nt, or past a right-hand side's active length)
// and truncation (outputs past Nt) are fused into the loads and stores.
#include "common.hpp"
#include "fft_common.hpp"
#include "kernels.hpp"

namespace p2o {

constexpr int kFftThreads = 256;

template <typename T> struct FftCap;
template <> struct FftCap<float> { static constexpr int cap = 3584; };   // complex tile entries per workgroup
template <> struct FftCap<double> { static constexpr int cap = 1792; };

// Tile element (bin n, series s) in LDS.  Rows are padded by one element:
// an odd row stride keeps the strided writes of the first Stockham passes
// (stride R rows) on distinct banks.
__device__ __forceinline__ int tix(int n, int s, int twsh) { return n * ((1 << twsh) + 1) + s; }

// One Stockham pass of radix R over a [M][TW] tile: butterfly j (of M/R)
// reads z[j + q M/R], applies twiddles e^{-2 pi i q k / (Ns R)} with
// k = j mod Ns, transforms, and writes z[(j / Ns) Ns R + k + p Ns].
template <typename T, int R, bool INV, int MAXV>
__device__ __forceinline__ void fft_pass(cplx<T>* buf, int twsh, int M, int Ns,
                                         const cplx<T>* __restrict__ tw, int L) {
    using Z = cplx<T>;
    constexpr int MAXBF = (MAXV + R - 1) / R;
    const int TWm = (1 << twsh) - 1;
    const int MR = M / R;
    const int nbf = MR << twsh;
    const int tstep = L / (Ns * R);
    // j / Ns by multiply-high: exact for j, Ns < 2^16
    const uint32_t mNs = Ns > 1 ? 0xFFFFFFFFu / (uint32_t)Ns + 1u : 0u;
    Z v[MAXBF][R];
#pragma unroll
    for (int u = 0; u < MAXBF; ++u) {
        const int bf = threadIdx.x + u * kFftThreads;
        if (bf < nbf) {
            const int s = bf & TWm;
            const int j = bf >> twsh;
            const int grp = Ns > 1 ? (int)__umulhi((uint32_t)j, mNs) : j;
            const int k = j - grp * Ns;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                Z a = buf[tix(j + q * MR, s, twsh)];
                if (q > 0 && k > 0) {
                    Z t = tw[q * k * tstep];
                    a = cmul(a, INV ? cconj(t) : t);
                }
                v[u][q] = a;
            }
            dft_small<T, R, INV>(v[u]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MAXBF; ++u) {
        const int bf = threadIdx.x + u * kFftThreads;
        if (bf < nbf) {
            const int s = bf & TWm;
            const int j = bf >> twsh;
            const int grp = Ns > 1 ? (int)__umulhi((uint32_t)j, mNs) : j;
            const int k = j - grp * Ns;
            const int base = grp * Ns * R + k;
#pragma unroll
            for (int p = 0; p < R; ++p) buf[tix(base + p * Ns, s, twsh)] = v[u][p];
        }
    }
    __syncthreads();
}

template <typename T, bool INV>
__device__ void fft_tile(cplx<T>* buf, int twsh, const FftPlan& pl, const cplx<T>* __restrict__ tw) {
    constexpr int MAXV = FftCap<T>::cap / kFftThreads;
    int Ns = 1;
    for (int p = 0; p < pl.npass; ++p) {
        const int R = pl.radix[p];
        switch (R) {
            case 2: fft_pass<T, 2, INV, MAXV>(buf, twsh, pl.M, Ns, tw, pl.L); break;
            case 3: fft_pass<T, 3, INV, MAXV>(buf, twsh, pl.M, Ns, tw, pl.L); break;
            case 4: fft_pass<T, 4, INV, MAXV>(buf, twsh, pl.M, Ns, tw, pl.L); break;
            case 5: fft_pass<T, 5, INV, MAXV>(buf, twsh, pl.M, Ns, tw, pl.L); break;
            case 7: fft_pass<T, 7, INV, MAXV>(buf, twsh, pl.M, Ns, tw, pl.L); break;
            default: fft_pass<T, 8, INV, MAXV>(buf, twsh, pl.M, Ns, tw, pl.L); break;
        }
        Ns *= R;
    }
}

// ---------------------------------------------------------------- real <-> half spectrum
// X[k] = (Z[k] + conj Z[M-k]) / 2 - (i/2) W^k (Z[k] - conj Z[M-k]), W = e^{-2 pi i / L},
// k = 0..M (Z is M-periodic).  Calls store(k, s, X).
template <typename T, typename Store>
__device__ __forceinline__ void r2c_post(const cplx<T>* buf, int twsh, int M,
                                         const cplx<T>* __restrict__ tw, Store&& store) {
    using Z = cplx<T>;
    const int TWm = (1 << twsh) - 1;
    for (int e = threadIdx.x; e < ((M + 1) << twsh); e += kFftThreads) {
        const int k = e >> twsh, s = e & TWm;
        const int k1 = (k == M) ? 0 : k;
        const int k2 = (k == 0) ? 0 : M - k;
        const Z a = buf[tix(k1, s, twsh)];
        const Z b = cconj(buf[tix(k2, s, twsh)]);
        const Z sum = cadd(a, b);
        const Z t = cmul(tw[k], csub(a, b));
        store(k, s, cmk<T>(T(0.5) * (sum.x + t.y), T(0.5) * (sum.y - t.x)));
    }
}

// Inverse of r2c_post on a tile holding X[0..M]: leaves Z[0..M-1] with
// Z[k] = E[k] + i O[k], E = (X[k] + conj X[M-k]) / 2,
// O = conj(W^k) (X[k] - conj X[M-k]) / 2.  Bins 0 and M are taken as real.
template <typename T>
__device__ __forceinline__ void c2r_pre(cplx<T>* buf, int twsh, int M, const cplx<T>* __restrict__ tw) {
    using Z = cplx<T>;
    const int TWm = (1 << twsh) - 1;
    auto one = [&](Z xa, Z xb, Z w) {
        const Z cb = cconj(xb);
        const Z E = cscale(cadd(xa, cb), T(0.5));
        const Z O = cscale(cmul(cconj(w), csub(xa, cb)), T(0.5));
        return cmk<T>(E.x - O.y, E.y + O.x);
    };
    for (int e = threadIdx.x; e < ((M / 2 + 1) << twsh); e += kFftThreads) {
        const int k = e >> twsh, s = e & TWm;
        const int kk = M - k;
        Z xk = buf[tix(k, s, twsh)];
        Z xkk = buf[tix(kk, s, twsh)];
        if (k == 0) { xk.y = T(0); xkk.y = T(0); }
        const Z zk = one(xk, xkk, tw[k]);
        if (k != 0 && kk != k) {
            const Z zkk = one(xkk, xk, tw[kk]);
            buf[tix(kk, s, twsh)] = zkk;
        }
        buf[tix(k, s, twsh)] = zk;
    }
}

// Copy the twiddle table e^{-2 pi i n / L} into LDS (callers synchronise).
template <typename T>
__device__ __forceinline__ void stage_twiddles(cplx<T>* tws, const cplx<T>* __restrict__ tw, int L) {
    for (int i = threadIdx.x; i < L; i += kFftThreads) tws[i] = tw[i];
}

// Load real series (zero past the active length) as z[n] = x[2n] + i x[2n+1].
template <typename T, typename TIN>
__device__ __forceinline__ void load_time(cplx<T>* buf, int twsh, int M, const TIN* __restrict__ src,
                                          long long t_stride, int S, int s0, int nt) {
    const int TWm = (1 << twsh) - 1;
    for (int e = threadIdx.x; e < (M << twsh); e += kFftThreads) {
        const int n = e >> twsh, s = e & TWm;
        const int col = s0 + s;
        T x0 = T(0), x1 = T(0);
        if (col < S) {
            const int t0 = 2 * n;
            if (t0 < nt) x0 = (T)src[(long long)t0 * t_stride + col];
            if (t0 + 1 < nt) x1 = (T)src[(long long)(t0 + 1) * t_stride + col];
        }
        buf[tix(n, s, twsh)] = cmk<T>(x0, x1);
    }
}

// Load a half spectrum X[0..M], summing `nparts` partial spectra in order.
// All of a thread's global loads of one partial are issued before any LDS
// store, so their latencies overlap instead of adding up.
template <typename T>
__device__ __forceinline__ void load_spec(cplx<T>* buf, int twsh, int M, const cplx<T>* __restrict__ src,
                                          long long f_stride, long long f_part, int nparts, int S, int s0) {
    using Z = cplx<T>;
    constexpr int MAXE = FftCap<T>::cap / kFftThreads;
    const int TWm = (1 << twsh) - 1;
    const int ne = (M + 1) << twsh;
    Z acc[MAXE];
#pragma unroll
    for (int u = 0; u < MAXE; ++u) acc[u] = cmk<T>(T(0), T(0));
    for (int q = 0; q < nparts; ++q) {
        Z v[MAXE];
#pragma unroll
        for (int u = 0; u < MAXE; ++u) {
            const int e = threadIdx.x + u * kFftThreads;
            const int k = e >> twsh, col = s0 + (e & TWm);
            v[u] = (e < ne && col < S) ? src[(long long)q * f_part + (long long)k * f_stride + col]
                                       : cmk<T>(T(0), T(0));
        }
#pragma unroll
        for (int u = 0; u < MAXE; ++u) acc[u] = cadd(acc[u], v[u]);
    }
#pragma unroll
    for (int u = 0; u < MAXE; ++u) {
        const int e = threadIdx.x + u * kFftThreads;
        if (e < ne) buf[tix(e >> twsh, e & TWm, twsh)] = acc[u];
    }
}

// Half spectra of a transformed tile to row[k * f_stride + s0 + s], zeros for
// series in [S, S_pad) (the tile holds zeros there), as complex values or,
// with io.quad (FP32 only), in quad BF16 hi/lo storage.
template <typename T>
__device__ __forceinline__ void store_half_spectra(const cplx<T>* buf, int twsh, int M, const cplx<T>* tw,
                                                   const SeriesIO& io, cplx<T>* row, int s0, float* amax_slot) {
    using Z = cplx<T>;
    if constexpr (sizeof(T) == sizeof(float)) {
        if (io.quad) {
            uint32_t* q = reinterpret_cast<uint32_t*>(row);
            r2c_post<T>(buf, twsh, M, tw, [&](int k, int s, Z X) {
                if (s0 + s < io.S_pad) store_quad(q + 2 * (long long)k * io.f_stride, s0 + s, X.x, X.y);
            });
            return;
        }
    }
    Z* dst = row + s0;
    float vmax = 0.f;
    r2c_post<T>(buf, twsh, M, tw, [&](int k, int s, Z X) {
        if (s0 + s < io.S_pad) {
            dst[(long long)k * io.f_stride + s] = X;
            if constexpr (sizeof(T) == sizeof(float)) vmax = fmaxf(vmax, fmaxf(fabsf(X.x), fabsf(X.y)));
        }
    });
    // FP16 matrix-core operands: each wavefront's largest |re|, |im|
    if constexpr (sizeof(T) == sizeof(float)) {
        if (amax_slot) wave_amax_store(vmax, amax_slot);
    }
}

__device__ __forceinline__ float* amax_slots_of(const SeriesIO& io, int outer, int tile) {
    return io.amax_part ? io.amax_part + (long long)outer * io.amax_slots + tile * (kFftThreads / 64) : nullptr;
}

// Right-hand-side scales from the wavefront maxima of one transform: block b
// reduces the `slots` maxima of outer index b and writes the power of two
// 2^(15 - ceil(log2 max)) (1 for an all-zero or non-finite maximum; the
// exponent is clamped to the FP32 range), so that max * scale lies in
// (2^14, 2^15]: every scaled value then fits FP16, and values far below the
// maximum keep an absolute precision of 2^-25 of the scaled unit.
__global__ void k_rhs_scale(const float* __restrict__ part, int slots, int stride, float* __restrict__ scale) {
    __shared__ float red[256];
    const float* p = part + (long long)blockIdx.x * stride;
    float v = 0.f;
    for (int i = threadIdx.x; i < slots; i += 256) v = fmaxf(v, p[i]);
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float a = red[0];
        float sc = 1.f;
        if (a > 0.f && a <= 3.0e38f) {
            int e;
            const float f = frexpf(a, &e);                 // a = f 2^e, f in [1/2, 1)
            const int c = f == 0.5f ? e - 1 : e;           // ceil(log2 a)
            sc = ldexpf(1.f, max(-126, min(126, 15 - c)));
        }
        scale[blockIdx.x] = sc;
    }
}

// ---------------------------------------------------------------- kernels
// r2c: time series [outer][t][col] -> half spectra [outer][k][col] (cols >= S zero-filled up to S_pad)
template <typename T, typename TIN>
__global__ __launch_bounds__(kFftThreads) void k_r2c(FftPlan pl, SeriesIO io, const TIN* __restrict__ in,
                                                     cplx<T>* __restrict__ out, const cplx<T>* __restrict__ twg,
                                                     int twsh, ItemMap im) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    using Z = cplx<T>;
    Z* buf = reinterpret_cast<Z*>(smem_raw);
    Z* tw = buf + (pl.M + 1) * ((1 << twsh) + 1);
    int tile, outer;
    if (!fft_item(im, tile, outer)) return;
    const int s0 = tile << twsh;
    const int nt = active_len(io, outer);
    stage_twiddles<T>(tw, twg, pl.L);
    load_time<T, TIN>(buf, twsh, pl.M, in + (long long)outer * io.t_outer, io.t_stride, io.S, s0, nt);
    __syncthreads();
    fft_tile<T, false>(buf, twsh, pl, tw);
    store_half_spectra<T>(buf, twsh, pl.M, tw, io, out + (long long)outer * io.f_outer, s0,
                          amax_slots_of(io, outer, tile));
}

// c2r: half spectra (sum of nparts partials) -> time series, truncated to Nt
// (and to the active length, zeros past it).  With EPI_MISFIT the stored
// value is w = (y - d_obs) / var and the FP64 sum of r * w over the tile
// goes to `partials[outer * ntiles + tile]`.
template <typename T, typename TOUT, int EPI>
__global__ __launch_bounds__(kFftThreads) void k_c2r(FftPlan pl, SeriesIO io, const cplx<T>* __restrict__ in,
                                                     TOUT* __restrict__ out, const cplx<T>* __restrict__ twg,
                                                     int twsh, MisfitArgs ma, ItemMap im) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    using Z = cplx<T>;
    Z* buf = reinterpret_cast<Z*>(smem_raw);
    Z* tw = buf + (pl.M + 1) * ((1 << twsh) + 1);
    int tile, outer;
    if (!fft_item(im, tile, outer)) return;
    const int s0 = tile << twsh;
    const int TWm = (1 << twsh) - 1;
    const int nt = active_len(io, outer);
    stage_twiddles<T>(tw, twg, pl.L);
    load_spec<T>(buf, twsh, pl.M, in + (long long)outer * io.f_outer, io.f_stride, io.f_part, io.nparts, io.S, s0);
    __syncthreads();
    c2r_pre<T>(buf, twsh, pl.M, tw);
    __syncthreads();
    fft_tile<T, true>(buf, twsh, pl, tw);
    const T inv = T(1) / T(pl.M);
    TOUT* dst = out + (long long)outer * io.t_outer;
    double acc = 0.0;
    for (int e = threadIdx.x; e < (pl.M << twsh); e += kFftThreads) {
        const int n = e >> twsh, s = e & TWm;
        const int col = s0 + s;
        if (col >= io.S) continue;
        const Z z = buf[tix(n, s, twsh)];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int t = 2 * n + h;
            if (t >= io.Nt) break;
            const T y = (h == 0 ? z.x : z.y) * inv;
            const long long off = (long long)t * io.t_stride + col;
            if constexpr (EPI == EPI_PLAIN) {
                dst[off] = (t < nt) ? (TOUT)y : TOUT(0);
            } else {
                const TOUT* dob = reinterpret_cast<const TOUT*>(ma.d_obs) + (long long)outer * io.t_outer;
                double r = 0.0, wv = 0.0;
                if (t < nt) {
                    const double var = ma.var_mode == 0 ? ma.var[0]
                                     : ma.var_mode == 1 ? ma.var[col]
                                                        : ma.var[(long long)t * io.S + col];
                    r = (double)y - (double)dob[off];
                    wv = r / var;
                    acc += r * wv;
                }
                dst[off] = (TOUT)wv;
            }
        }
    }
    if constexpr (EPI == EPI_MISFIT) {
        __syncthreads();                       // LDS tile is free now
        double* red = reinterpret_cast<double*>(smem_raw);
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = kFftThreads / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) ma.partials[(long long)outer * im.ntiles + tile] = red[0];
    }
}

// Truncate-and-repad between the adjoint and forward passes of F F^*:
// half spectra (sum of partials) -> time series -> keep t < active length
// -> half spectra again, written over partial 0 of the input (every
// workgroup reads its whole tile before it writes; in quad storage a tile
// must span whole groups of 4 series).
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_project(FftPlan pl, SeriesIO io, cplx<T>* in_out,
                                                         const cplx<T>* __restrict__ twg, int twsh, ItemMap im) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    using Z = cplx<T>;
    Z* buf = reinterpret_cast<Z*>(smem_raw);
    Z* tw = buf + (pl.M + 1) * ((1 << twsh) + 1);
    int tile, outer;
    if (!fft_item(im, tile, outer)) return;
    const int s0 = tile << twsh;
    const int TWm = (1 << twsh) - 1;
    const int nt = active_len(io, outer);
    stage_twiddles<T>(tw, twg, pl.L);
    Z* base = in_out + (long long)outer * io.f_outer;
    load_spec<T>(buf, twsh, pl.M, base, io.f_stride, io.f_part, io.nparts, io.S, s0);
    __syncthreads();
    c2r_pre<T>(buf, twsh, pl.M, tw);
    __syncthreads();
    fft_tile<T, true>(buf, twsh, pl, tw);
    const T inv = T(1) / T(pl.M);
    for (int e = threadIdx.x; e < (pl.M << twsh); e += kFftThreads) {
        const int n = e >> twsh, i = tix(n, e & TWm, twsh);
        Z z = buf[i];
        z.x = (2 * n < nt) ? z.x * inv : T(0);
        z.y = (2 * n + 1 < nt) ? z.y * inv : T(0);
        buf[i] = z;
    }
    __syncthreads();
    fft_tile<T, false>(buf, twsh, pl, tw);
    store_half_spectra<T>(buf, twsh, pl.M, tw, io, base, s0, amax_slots_of(io, outer, tile));
}

// Fixed-order sum of the misfit partials: misfit[b] = 1/2 sum_x partials[b][x].
__global__ void k_misfit_reduce(const double* __restrict__ partials, int nper, double* __restrict__ misfit,
                                int nrhs) {
    __shared__ double red[256];
    const int b = blockIdx.x;
    if (b >= nrhs) return;
    double acc = 0.0;
    for (int x = threadIdx.x; x < nper; x += 256) acc += partials[(long long)b * nper + x];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) misfit[b] = 0.5 * red[0];
}

// ---------------------------------------------------------------- loading the spectrum
// Twiddles e^{-2 pi i n / L}, n < L, in FP64 (sincospi takes the angle in
// units of pi, so the only rounding before it is that of 2n/L), also
// rounded to FP32.
__global__ void k_twiddle(double2* __restrict__ tw64, float2* __restrict__ tw32, int L) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= L) return;
    double s, c;
    sincospi(-(2.0 * (double)n) / (double)L, &s, &c);
    tw64[n] = make_double2(c, s);
    tw32[n] = make_float2((float)c, (float)s);
}

__device__ __forceinline__ int quant_exponent(float amax, int prec) {
    if (!(amax > 0.0f)) return 0;
    int ex;
    const float f = frexpf(amax, &ex);          // amax = f 2^ex, f in [1/2, 1)
    const int clog2 = (f == 0.5f) ? ex - 1 : ex; // ceil(log2 amax)
    int e = (prec == kFP16 ? 15 : 0) - clog2;
    e = e < -126 ? -126 : (e > 126 ? 126 : e);
    return e;
}

// Transform columns of the time-domain blocks, all rows in [row0, row0+rows).
// PASS 0: per-(bin, scale block) maximum magnitude of real and imaginary
// parts, accumulated as float bits with atomicMax into `amax` (exact and
// order independent), and a non-finite flag.  PASS 1: round and store.
template <typename TIN, int P, int PASS>
__global__ __launch_bounds__(kFftThreads) void k_load(FftPlan pl, LoadArgs la, const TIN* __restrict__ in,
                                                      const double2* __restrict__ twg, int twsh, ItemMap im) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    using Z = double2;
    Z* buf = reinterpret_cast<Z*>(smem_raw);
    Z* tw = buf + (pl.M + 1) * ((1 << twsh) + 1);
    unsigned* lmax = reinterpret_cast<unsigned*>(tw + pl.L);
    int tile, rgroup;
    if (!fft_item(im, tile, rgroup)) return;
    stage_twiddles<double>(tw, twg, pl.L);
    const int s0 = tile << twsh;
    const int TWm = (1 << twsh) - 1;
    const int blk = (int)((la.col0 + s0) / kScaleBlock);
    bool bad = false;
    if constexpr (PASS == 0) {
        for (int k = threadIdx.x; k <= pl.M; k += kFftThreads) lmax[k] = 0u;
    }
    const int r0 = rgroup * la.rows_per_wg;
    const int r1 = min(la.Nd, r0 + la.rows_per_wg);
    for (int row = r0; row < r1; ++row) {
        const TIN* src = in + (long long)row * la.ncols;
        load_time<double, TIN>(buf, twsh, pl.M, src, la.t_stride, la.ncols, s0, la.Nt);
        if constexpr (PASS == 0 || !Fmt<P>::scaled) {
            for (int e = threadIdx.x; e < (pl.M << twsh); e += kFftThreads) {
                const double2 z = buf[tix(e >> twsh, e & TWm, twsh)];
                bad |= !isfinite(z.x) || !isfinite(z.y);
            }
        }
        __syncthreads();
        fft_tile<double, false>(buf, twsh, pl, tw);
        r2c_post<double>(buf, twsh, pl.M, tw, [&](int k, int s, Z X) {
            const long long col = la.col0 + s0 + s;
            if constexpr (PASS == 0) {
                if (s0 + s < la.ncols) {
                    const float m = (float)fmax(fabs(X.x), fabs(X.y));
                    atomicMax(&lmax[k], __float_as_uint(m));
                }
            } else {
                if (s0 + s >= la.ncols) return;
                const long long off = ((long long)k * la.Nd + row) * la.pitch + col;
                if constexpr (P == kFP64) {
                    reinterpret_cast<double2*>(la.fhat)[off] = X;
                } else if constexpr (P == kFP32) {
                    reinterpret_cast<float2*>(la.fhat)[off] = make_float2((float)X.x, (float)X.y);
                } else {
                    const float am = __uint_as_float(reinterpret_cast<const unsigned*>(la.scales)[k * la.nblk + blk]);
                    const int ex = quant_exponent(am, P);
                    const float re = f64_to_f32_odd(ldexp(X.x, ex));
                    const float im = f64_to_f32_odd(ldexp(X.y, ex));
                    uint32_t q;
                    if constexpr (P == kBF16) q = f32_to_bf16_rne(re) | (f32_to_bf16_rne(im) << 16);
                    else q = f32_to_f16_rne(re) | (f32_to_f16_rne(im) << 16);
                    reinterpret_cast<uint32_t*>(la.fhat)[off] = q;
                }
            }
        });
        __syncthreads();
    }
    if constexpr (PASS == 0) {
        for (int k = threadIdx.x; k <= pl.M; k += kFftThreads)
            atomicMax(reinterpret_cast<unsigned*>(la.scales) + k * la.nblk + blk, lmax[k]);
    }
    if (bad) atomicOr(la.flag, 1u);
}

// Zero (PASS 0 start) the amax slots of scale blocks [blk0, blk1), or turn
// them into dequantisation multipliers 2^-e, or set multipliers to 1.
__global__ void k_scales(float* __restrict__ scales, int nfreq, int nblk, int blk0, int blk1, int mode, int prec) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nb = blk1 - blk0;
    if (i >= nfreq * nb) return;
    const int k = i / nb, b = blk0 + i % nb;
    float* p = scales + (long long)k * nblk + b;
    if (mode == 0) *p = 0.0f;
    else if (mode == 1) *p = ldexpf(1.0f, -quant_exponent(*p, prec));
    else *p = 1.0f;
}

// Zero-fill of the padding columns [Nm, pitch) of every stored row.
__global__ void k_zero_pad(uint8_t* __restrict__ fhat, long long rows, int pitch, int Nm, int bytes) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int w = (pitch - Nm) * bytes;
    if (w <= 0 || i >= rows * w) return;
    const long long r = i / w;
    fhat[r * (long long)pitch * bytes + (long long)Nm * bytes + (i % w)] = 0;
}

// ---------------------------------------------------------------- host launchers
// Tile width TW (a power of two, at most 32 series): the largest that keeps
// the tile plus the twiddle table within 48 KiB of LDS, so that three or four
// workgroups share a CU.
constexpr size_t kFftLdsTarget = 48 * 1024;

static size_t fft_lds(int M, int twsh, size_t zbytes) {
    return ((size_t)(M + 1) * (((size_t)1 << twsh) + 1) + (size_t)(2 * M)) * zbytes;
}

int fft_tile_shift(int M, bool f64) {
    const size_t z = f64 ? sizeof(double2) : sizeof(float2);
    const int cap = f64 ? FftCap<double>::cap : FftCap<float>::cap;
    for (int sh = 5; sh >= 0; --sh)
        if (fft_lds(M, sh, z) <= kFftLdsTarget && ((M + 1) << sh) <= cap) return sh;
    return -1;
}

// The loader also keeps one running maximum per bin in LDS.
static size_t load_lds(int M, int sh) { return fft_lds(M, sh, sizeof(double2)) + (size_t)(M + 1) * sizeof(unsigned); }

int load_tile_shift(int M) {
    for (int sh = 5; sh >= 0; --sh)
        if (load_lds(M, sh) <= 65536 && ((M + 1) << sh) <= FftCap<double>::cap) return sh;
    return -1;
}

static ItemMap item_map(int S, int sh, int outer) {
    ItemMap im;
    im.ntiles = (S + (1 << sh) - 1) >> sh;
    im.items = im.ntiles * outer;
    im.Q = (im.items + 7) / 8;
    return im;
}

hipError_t launch_twiddle(void* tw64, void* tw32, int L, hipStream_t st) {
    hipLaunchKernelGGL(k_twiddle, dim3((L + 255) / 256), dim3(256), 0, st,
                       (double2*)tw64, (float2*)tw32, L);
    return hipGetLastError();
}

// After a transform that recorded wavefront maxima: the per-outer scales,
// from the slots of its tiles (tile shift sh; four wavefronts per tile on
// the runtime-length kernels, fixed_tile_waves on the compiled-length ones).
static hipError_t rhs_scales(const FftPlan& pl, bool f64, const SeriesIO& io, int sh, hipError_t err,
                             hipStream_t st) {
    if (err != hipSuccess || !io.amax_part || io.outer_count == 0) return err;
    static_assert(kFftThreads == 256, "four wavefronts per runtime-length tile");
    const int used = ((io.S_pad + (1 << sh) - 1) >> sh) * fixed_tile_waves(f64, pl, sh);
    hipLaunchKernelGGL(k_rhs_scale, dim3(io.outer_count), dim3(256), 0, st, (const float*)io.amax_part, used,
                       io.amax_slots, io.rhs_scale);
    return hipGetLastError();
}

// Wavefront-maximum slots per outer index that the transforms of S_pad
// series need at most (tiles of at least 4 series, 256-thread workgroups).
int fft_amax_slots(int S_pad) { return (S_pad + 3) / 4 * (kFftThreads / 64); }

// Wide tile shift for a transform of S series (when the compiled-length
// kernels have one), else -1.  A transform that takes it reports the shift
// it used, so that the per-tile maxima are read back with the same tiling.
static int wide_shift(bool f64, const FftPlan& pl, int S) { return S >= kWideSeries ? fixed_wide_shift(f64, pl) : -1; }

static hipError_t r2c_transform(bool f64, bool in_f64, const FftPlan& pl, const SeriesIO& io, const void* in,
                                void* out, const void* tw, hipStream_t st, int* sh_used) {
    hipError_t err;
    const int wsh = wide_shift(f64, pl, io.S_pad);
    *sh_used = wsh;
    if (wsh >= 0 && launch_fixed_r2c(f64, in_f64, pl, io, in, out, tw, wsh, st, &err)) return err;
    const int sh = fft_tile_shift(pl.M, f64);
    *sh_used = sh;
    if (launch_fixed_r2c(f64, in_f64, pl, io, in, out, tw, sh, st, &err)) return err;
    const ItemMap im = item_map(io.S_pad, sh, io.outer_count);
    if (io.amax_part && (long long)im.ntiles * (kFftThreads / 64) > io.amax_slots) return hipErrorInvalidValue;
    dim3 grid(8 * im.Q);
    if (f64) {
        const size_t lds = fft_lds(pl.M, sh, sizeof(double2));
        if (in_f64) hipLaunchKernelGGL((k_r2c<double, double>), grid, dim3(kFftThreads), lds, st, pl, io, (const double*)in, (double2*)out, (const double2*)tw, sh, im);
        else hipLaunchKernelGGL((k_r2c<double, float>), grid, dim3(kFftThreads), lds, st, pl, io, (const float*)in, (double2*)out, (const double2*)tw, sh, im);
    } else {
        const size_t lds = fft_lds(pl.M, sh, sizeof(float2));
        hipLaunchKernelGGL((k_r2c<float, float>), grid, dim3(kFftThreads), lds, st, pl, io, (const float*)in, (float2*)out, (const float2*)tw, sh, im);
    }
    return hipGetLastError();
}

hipError_t launch_r2c(bool f64, bool in_f64, const FftPlan& pl, const SeriesIO& io, const void* in, void* out,
                      const void* tw, hipStream_t st) {
    int sh = 0;
    const hipError_t err = r2c_transform(f64, in_f64, pl, io, in, out, tw, st, &sh);
    return rhs_scales(pl, f64, io, sh, err, st);
}

hipError_t launch_c2r(bool f64, const FftPlan& pl, const SeriesIO& io, const void* in, void* out, const void* tw,
                      const void* d_obs, const double* var, int var_mode, double* partials, hipStream_t st) {
    hipError_t err;
    // the misfit epilogue's partials are counted per tile of the runtime
    // tile shift (c2r_grid_x), so it never takes wide tiles
    const int wsh = d_obs ? -1 : wide_shift(f64, pl, io.S);
    if (wsh >= 0 && launch_fixed_c2r(f64, pl, io, in, out, tw, wsh, d_obs, var, var_mode, partials, st, &err)) return err;
    const int sh = fft_tile_shift(pl.M, f64);
    if (launch_fixed_c2r(f64, pl, io, in, out, tw, sh, d_obs, var, var_mode, partials, st, &err)) return err;
    const ItemMap im = item_map(io.S, sh, io.outer_count);
    dim3 grid(8 * im.Q);
    MisfitArgs ma{d_obs, var, var_mode, partials};
    const bool mis = d_obs != nullptr;
    if (f64) {
        size_t lds = fft_lds(pl.M, sh, sizeof(double2));
        if (lds < kFftThreads * sizeof(double)) lds = kFftThreads * sizeof(double);
        if (mis) hipLaunchKernelGGL((k_c2r<double, double, EPI_MISFIT>), grid, dim3(kFftThreads), lds, st, pl, io, (const double2*)in, (double*)out, (const double2*)tw, sh, ma, im);
        else hipLaunchKernelGGL((k_c2r<double, double, EPI_PLAIN>), grid, dim3(kFftThreads), lds, st, pl, io, (const double2*)in, (double*)out, (const double2*)tw, sh, ma, im);
    } else {
        size_t lds = fft_lds(pl.M, sh, sizeof(float2));
        if (lds < kFftThreads * sizeof(double)) lds = kFftThreads * sizeof(double);
        if (mis) hipLaunchKernelGGL((k_c2r<float, float, EPI_MISFIT>), grid, dim3(kFftThreads), lds, st, pl, io, (const float2*)in, (float*)out, (const float2*)tw, sh, ma, im);
        else hipLaunchKernelGGL((k_c2r<float, float, EPI_PLAIN>), grid, dim3(kFftThreads), lds, st, pl, io, (const float2*)in, (float*)out, (const float2*)tw, sh, ma, im);
    }
    return hipGetLastError();
}

int c2r_grid_x(const FftPlan& pl, bool f64, int S) {
    const int sh = fft_tile_shift(pl.M, f64);
    return (S + (1 << sh) - 1) >> sh;
}

static hipError_t project_transform(bool f64, const FftPlan& pl, const SeriesIO& io, void* in_out, const void* tw,
                                    hipStream_t st, int* sh_used) {
    hipError_t err;
    const int wsh = wide_shift(f64, pl, io.S_pad);
    *sh_used = wsh;
    if (wsh >= 0 && launch_fixed_project(f64, pl, io, in_out, tw, wsh, st, &err)) return err;
    const int sh = fft_tile_shift(pl.M, f64);
    *sh_used = sh;
    if (launch_fixed_project(f64, pl, io, in_out, tw, sh, st, &err)) return err;
    const ItemMap im = item_map(io.S_pad, sh, io.outer_count);
    if (io.amax_part && (long long)im.ntiles * (kFftThreads / 64) > io.amax_slots) return hipErrorInvalidValue;
    dim3 grid(8 * im.Q);
    if (f64) hipLaunchKernelGGL((k_project<double>), grid, dim3(kFftThreads), fft_lds(pl.M, sh, sizeof(double2)), st, pl, io, (double2*)in_out, (const double2*)tw, sh, im);
    else hipLaunchKernelGGL((k_project<float>), grid, dim3(kFftThreads), fft_lds(pl.M, sh, sizeof(float2)), st, pl, io, (float2*)in_out, (const float2*)tw, sh, im);
    return hipGetLastError();
}

bool launch_project_half(const FftPlan& pl, const SeriesIO& io, void* in_out, const void* tw, const float* sx,
                         const float* sy, hipStream_t st, hipError_t* err) {
    // FP16 pairs: a 16-series tile's bin rows are 64 bytes whichever the
    // workgroup size; at M = 420 the re-pad on FP16 pairs measured 3 % slower
    // on the wide tiles than on 8-series ones, so it keeps those there
    const int wsh = pl.M == 420 ? -1 : wide_shift(false, pl, io.S_pad);
    if (wsh >= 0 && launch_fixed_project_h(pl, io, in_out, tw, wsh, sx, sy, st, err)) return true;
    return launch_fixed_project_h(pl, io, in_out, tw, fft_tile_shift(pl.M, false), sx, sy, st, err);
}

hipError_t launch_project(bool f64, const FftPlan& pl, const SeriesIO& io, void* in_out, const void* tw,
                          hipStream_t st) {
    int sh = 0;
    const hipError_t err = project_transform(f64, pl, io, in_out, tw, st, &sh);
    return rhs_scales(pl, f64, io, sh, err, st);
}

hipError_t launch_misfit_reduce(const double* partials, int nper, double* misfit, int nrhs, hipStream_t st) {
    hipLaunchKernelGGL(k_misfit_reduce, dim3(nrhs), dim3(256), 0, st, partials, nper, misfit, nrhs);
    return hipGetLastError();
}

template <typename TIN, int P>
static void load_pass(int pass, dim3 grid, size_t lds, hipStream_t st, const FftPlan& pl, const LoadArgs& la,
                      const void* in, const void* tw, int sh, ItemMap im) {
    if (pass == 0) hipLaunchKernelGGL((k_load<TIN, P, 0>), grid, dim3(kFftThreads), lds, st, pl, la, (const TIN*)in, (const double2*)tw, sh, im);
    else hipLaunchKernelGGL((k_load<TIN, P, 1>), grid, dim3(kFftThreads), lds, st, pl, la, (const TIN*)in, (const double2*)tw, sh, im);
}

hipError_t launch_load(int prec, bool in_f64, const FftPlan& pl, const LoadArgs& la, const void* in,
                       const void* tw64, hipStream_t st) {
    const int sh = load_tile_shift(pl.M);
    if (sh < 0) return hipErrorInvalidValue;
    const ItemMap im = item_map(la.ncols, sh, (la.Nd + la.rows_per_wg - 1) / la.rows_per_wg);
    dim3 grid(8 * im.Q);
    const size_t lds = load_lds(pl.M, sh);
    const int nb0 = (int)(la.col0 / kScaleBlock);
    const int nb1 = (int)((la.col0 + la.ncols + kScaleBlock - 1) / kScaleBlock);
    const int nfreq = pl.M + 1;
    const int ns = nfreq * (nb1 - nb0);
    const bool scaled = prec == kBF16 || prec == kFP16;
    if (scaled) {
        hipLaunchKernelGGL(k_scales, dim3((ns + 255) / 256), dim3(256), 0, st, la.scales, nfreq, la.nblk, nb0, nb1, 0, prec);
    } else {
        hipLaunchKernelGGL(k_scales, dim3((ns + 255) / 256), dim3(256), 0, st, la.scales, nfreq, la.nblk, nb0, nb1, 2, prec);
    }
    for (int pass = scaled ? 0 : 1; pass < 2; ++pass) {
        switch (prec) {
            case kFP64: in_f64 ? load_pass<double, kFP64>(pass, grid, lds, st, pl, la, in, tw64, sh, im) : load_pass<float, kFP64>(pass, grid, lds, st, pl, la, in, tw64, sh, im); break;
            case kFP32: in_f64 ? load_pass<double, kFP32>(pass, grid, lds, st, pl, la, in, tw64, sh, im) : load_pass<float, kFP32>(pass, grid, lds, st, pl, la, in, tw64, sh, im); break;
            case kBF16: in_f64 ? load_pass<double, kBF16>(pass, grid, lds, st, pl, la, in, tw64, sh, im) : load_pass<float, kBF16>(pass, grid, lds, st, pl, la, in, tw64, sh, im); break;
            default: in_f64 ? load_pass<double, kFP16>(pass, grid, lds, st, pl, la, in, tw64, sh, im) : load_pass<float, kFP16>(pass, grid, lds, st, pl, la, in, tw64, sh, im); break;
        }
    }
    if (scaled) {
        hipLaunchKernelGGL(k_scales, dim3((ns + 255) / 256), dim3(256), 0, st, la.scales, nfreq, la.nblk, nb0, nb1, 1, prec);
    }
    return hipGetLastError();
}

hipError_t launch_zero_pad(void* fhat, long long rows, int pitch, int Nm, int bytes, hipStream_t st) {
    const long long n = rows * (long long)(pitch - Nm) * bytes;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_pad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (uint8_t*)fhat, rows, pitch, Nm, bytes);
    return hipGetLastError();
}

}  // namespace p2o
