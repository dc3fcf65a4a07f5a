// Shared device-side definitions: complex arithmetic, storage formats of the
// Fourier blocks, and the launch descriptors passed from the host plan.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace p2o {

constexpr int kScaleBlock = 4096;   // columns per power-of-two scale block
constexpr int kMaxPasses = 16;

// ---------------------------------------------------------------- complex
template <typename T> struct cvec;
template <> struct cvec<float> { using type = float2; };
template <> struct cvec<double> { using type = double2; };
template <typename T> using cplx = typename cvec<T>::type;

template <typename T>
__device__ __forceinline__ cplx<T> cmk(T re, T im) { cplx<T> z; z.x = re; z.y = im; return z; }
template <typename Z>
__device__ __forceinline__ Z cadd(Z a, Z b) { a.x += b.x; a.y += b.y; return a; }
template <typename Z>
__device__ __forceinline__ Z csub(Z a, Z b) { a.x -= b.x; a.y -= b.y; return a; }
template <typename Z>
__device__ __forceinline__ Z cmul(Z a, Z b) {
    Z r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
template <typename Z>
__device__ __forceinline__ Z cconj(Z a) { a.y = -a.y; return a; }
template <typename Z, typename T>
__device__ __forceinline__ Z cscale(Z a, T s) { a.x *= s; a.y *= s; return a; }

// ---------------------------------------------------------------- storage
// Storage formats of one complex Fourier-block entry.  Every format keeps
// the real part first.  A lane moves 32 bytes of a row per access, so the
// number of complex entries per lane (V) depends on the format.
enum Prec : int { kFP64 = 0, kFP32 = 1, kBF16 = 2, kFP16 = 3 };

template <int P> struct Fmt;
template <> struct Fmt<kFP64> { using CT = double; static constexpr int bytes = 16; static constexpr int V = 2; static constexpr bool scaled = false; };
template <> struct Fmt<kFP32> { using CT = float;  static constexpr int bytes = 8;  static constexpr int V = 4; static constexpr bool scaled = false; };
template <> struct Fmt<kBF16> { using CT = float;  static constexpr int bytes = 4;  static constexpr int V = 8; static constexpr bool scaled = true; };
template <> struct Fmt<kFP16> { using CT = float;  static constexpr int bytes = 4;  static constexpr int V = 8; static constexpr bool scaled = true; };

struct Raw32 { uint4 a, b; };   // 32 bytes as eight dwords

__device__ __forceinline__ float bf16lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ float f16lo(uint32_t w) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
}
__device__ __forceinline__ float f16hi(uint32_t w) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}

// Unpack the 32 bytes a lane loaded into V complex entries (re[], im[]).
template <int P>
__device__ __forceinline__ void unpack(const Raw32& r, typename Fmt<P>::CT* re, typename Fmt<P>::CT* im) {
    const uint32_t w[8] = {r.a.x, r.a.y, r.a.z, r.a.w, r.b.x, r.b.y, r.b.z, r.b.w};
    if constexpr (P == kFP64) {
        re[0] = __hiloint2double(w[1], w[0]); im[0] = __hiloint2double(w[3], w[2]);
        re[1] = __hiloint2double(w[5], w[4]); im[1] = __hiloint2double(w[7], w[6]);
    } else if constexpr (P == kFP32) {
#pragma unroll
        for (int v = 0; v < 4; ++v) { re[v] = __uint_as_float(w[2 * v]); im[v] = __uint_as_float(w[2 * v + 1]); }
    } else if constexpr (P == kBF16) {
#pragma unroll
        for (int v = 0; v < 8; ++v) { re[v] = bf16lo(w[v]); im[v] = bf16hi(w[v]); }
    } else {
#pragma unroll
        for (int v = 0; v < 8; ++v) { re[v] = f16lo(w[v]); im[v] = f16hi(w[v]); }
    }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// 32-byte streaming load (non-temporal: the spectrum is read once per call).
// 32 bytes of a lane as two 16-byte halves 1 KB apart (half h only if lh):
// with lane L at base + 16 L, each load instruction of a wavefront covers one
// contiguous kilobyte, i.e. whole cache lines.
__device__ __forceinline__ Raw32 load32_split(const void* p, bool l0, bool l1) {
    const u32x4* q = reinterpret_cast<const u32x4*>(p);
    u32x4 a = {0u, 0u, 0u, 0u}, b = {0u, 0u, 0u, 0u};
    if (l0) a = __builtin_nontemporal_load(q);
    if (l1) b = __builtin_nontemporal_load(q + 64);
    Raw32 r;
    r.a = make_uint4(a.x, a.y, a.z, a.w);
    r.b = make_uint4(b.x, b.y, b.z, b.w);
    return r;
}

// Streaming stores (non-temporal: written through without keeping the
// lines), for outputs far larger than the caches.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4_nt __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_nt(float2* p, float2 v) {
    __builtin_nontemporal_store((u32x2){__float_as_uint(v.x), __float_as_uint(v.y)}, reinterpret_cast<u32x2*>(p));
}
__device__ __forceinline__ void store_nt(float4* p, float4 v) {
    __builtin_nontemporal_store((f32x4_nt){v.x, v.y, v.z, v.w}, reinterpret_cast<f32x4_nt*>(p));
}
__device__ __forceinline__ void store_nt(uint2* p, uint2 v) {
    __builtin_nontemporal_store((u32x2){v.x, v.y}, reinterpret_cast<u32x2*>(p));
}
__device__ __forceinline__ void store_nt(uint32_t* p, uint32_t v) { __builtin_nontemporal_store(v, p); }

__device__ __forceinline__ Raw32 load32(const void* p) {
    const u32x4* q = reinterpret_cast<const u32x4*>(p);
    const u32x4 a = __builtin_nontemporal_load(q);
    const u32x4 b = __builtin_nontemporal_load(q + 1);
    Raw32 r;
    r.a = make_uint4(a.x, a.y, a.z, a.w);
    r.b = make_uint4(b.x, b.y, b.z, b.w);
    return r;
}

// ---------------------------------------------------------------- rounding
// Round a double to float with round-to-odd: the float nearest below or
// above in magnitude, whichever has an odd last bit, unless exact.  A later
// round-to-nearest-even to any format with at most 22 significand bits then
// equals a single correct rounding of the double (Boldo & Melquiond,
// "Emulation of FMA and correctly rounded sums: proved algorithms using
// rounding to odd", IEEE TC 2008).
__device__ __forceinline__ float f64_to_f32_odd(double x) {
    float f = (float)x;
    double back = (double)f;
    if (back != x) {
        uint32_t u = __float_as_uint(f);
        if (fabs(back) > fabs(x)) u -= 1u;    // step back toward zero
        u |= 1u;
        f = __uint_as_float(u);
    }
    return f;
}

__device__ __forceinline__ uint32_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

// Two values rounded to BF16 (nearest even) in one word, a in the low half
// (one v_cvt_pk_bf16_f32 on gfx950).
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16_rne(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{a, b}, bf16x2_t));
}

// x = hi + lo with hi, lo BF16 (round to nearest even); the raw 16-bit codes.
__device__ __forceinline__ void split_bf16(float x, uint32_t& hi, uint32_t& lo) {
    hi = f32_to_bf16_rne(x);
    lo = f32_to_bf16_rne(x - __uint_as_float(hi << 16));
}

// "Quad" storage of a complex FP32 series as BF16 hi/lo pairs, the operand
// form of the matrix-core products: each group of 4 consecutive values takes
// 32 bytes, first the 4 hi words then the 4 lo words, a word holding
// (re, im) with re in the low half.  Same footprint as complex FP32; the
// series must start at a multiple of 4 values.  Stores value c of the series
// whose first word is q.
__device__ __forceinline__ void store_quad(uint32_t* q, long long c, float re, float im) {
    const uint32_t hi = pack_bf16_rne(re, im);
    const uint32_t lo = pack_bf16_rne(re - __uint_as_float(hi << 16), im - __uint_as_float(hi & 0xffff0000u));
    uint32_t* g = q + 8 * (c >> 2) + (c & 3);
    g[0] = hi;
    g[4] = lo;
}

__device__ __forceinline__ uint32_t f32_to_f16_rne(float f) {
    _Float16 h = (_Float16)f;
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
}

// ---------------------------------------------------------------- launch descriptors
struct FftPlan {
    int M;          // complex transform length, L / 2
    int L;          // circulant length
    int npass;
    int radix[kMaxPasses];
    int fixed;      // nonzero: use the kernels compiled for this M when there are any
};

// Addressing of a batch of real time series and their half spectra.
// Series are contiguous ("columns"); `outer` indexes right-hand sides (or,
// for loading, rows of the blocks).  Strides are in elements.
struct SeriesIO {
    long long t_stride;      // time-domain: step between time steps
    long long t_outer;       // time-domain: step between outer indices
    long long f_stride;      // frequency-domain: step between bins
    long long f_outer;       // frequency-domain: step between outer indices
    long long f_part;        // frequency-domain: step between partial sums
    int nparts;              // partial sums to add when reading a spectrum
    int S;                   // live series per outer index
    int S_pad;               // series written in the frequency domain (zeros past S)
    int quad;                // FP32 spectra written in quad BF16 hi/lo storage
    int Nt;                  // time steps
    int outer_count;
    const int* nt_active;    // per outer index, or nullptr
    // Right-hand-side scales of the FP16 matrix-core products (FP32 spectra
    // only, or nullptr): the producing transform writes the largest |re|,
    // |im| it stores per (outer index, tile, wavefront) to amax_part (at most
    // amax_slots slots per outer index), then rhs_scale[outer] receives the
    // power of two that maps that outer index's maximum into (2^14, 2^15].
    float* amax_part;
    float* rhs_scale;
    int amax_slots;
};

// Largest |re|, |im| of a wavefront's values, written by lane 0 to slot[wave].
__device__ __forceinline__ void wave_amax_store(float v, float* slot) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = v;
}

}  // namespace p2o
