// Batched real FFTs along time, compiled for fixed transform lengths.
//
// These compute what the runtime-length kernels in fft.hip compute (the
// circulant embedding of section 4: a tile of TW adjacent series x all bins
// in LDS as [bin][series], each real series of length L = 2M transformed as
// one complex series of length M, Stockham passes in place, zero padding and
// truncation fused into the loads and stores), with M, the tile width and
// the radix sequence known to the compiler.  That removes most of the
// integer work of the runtime-length passes:
//  - every LDS address of a pass is a per-thread base plus an instruction
//    immediate, and butterfly indices are divisions by constants;
//  - each pass reads its twiddles w[k][q] = e^{-2 pi i q k / (Ns R)} from a
//    table laid out in the order a butterfly uses them;
//  - the forward transform's first pass takes its inputs straight from the
//    time series, and the inverse transform's last pass writes its outputs
//    straight to them;
//  - in the truncate-and-repad kernel the inverse transform runs its radices
//    in reverse order, so that its last pass and the forward transform's
//    first pass cover the same index sets: both passes and the truncation
//    between them run on registers;
//  - the real-transform pre and post steps take bins k and M - k together
//    (they share their inputs, and W^(M-k) = -conj(W^k));
//  - workgroups are persistent (a grid of resident workgroups loops over the
//    tiles), so the twiddle tables are staged once per workgroup.
// Transform lengths without a compiled kernel use the runtime-length ones.
#include <algorithm>
#include <utility>

#include "common.hpp"
#include "fft_common.hpp"
#include "kernels.hpp"

namespace p2o {
namespace {


// M factored greedily over 8, 4, 2, 3, 5, 7 (as the plan does), in that order
// or reversed.  ns: product of the radices of the earlier passes; toff: first
// entry of the pass's twiddles in its table (the table has M - 1 entries).
struct RadixSeq {
    int n;
    int r[kMaxPasses];
    int ns[kMaxPasses];
    int toff[kMaxPasses];
};

constexpr RadixSeq radix_seq(int M, bool reversed) {
    RadixSeq f{};
    const int order[6] = {8, 4, 2, 3, 5, 7};
    int fac[kMaxPasses] = {};
    int n = 0, m = M;
    for (int i = 0; i < 6; ++i)
        while (m % order[i] == 0 && n < kMaxPasses) {
            fac[n++] = order[i];
            m /= order[i];
        }
    int ns = 1, off = 0;
    for (int p = 0; p < n; ++p) {
        const int r = reversed ? fac[n - 1 - p] : fac[p];
        f.r[p] = r;
        f.ns[p] = ns;
        f.toff[p] = off;
        off += ns * (r - 1);
        ns *= r;
    }
    f.n = n;
    return f;
}

template <int M, int SH, int NT>
struct Geo {
    static constexpr int TW = 1 << SH;             // series per tile
    static constexpr int RS = TW + 1;              // LDS row stride in complex entries (odd: spreads banks)
    static constexpr int JS = NT >> SH;            // bins (or butterflies) per sweep of the workgroup
    static constexpr RadixSeq FWD = radix_seq(M, false);
    static constexpr RadixSeq REV = radix_seq(M, true);
    static constexpr int NP = FWD.n;
    static constexpr int NPAIR = M / 2 + 1;        // bin pairs (k, M - k), k = 0 .. M / 2
    static constexpr int TILE = (M + 1) * RS;      // complex entries of the tile (bins 0 .. M)
    static_assert(M % 2 == 0 && NP >= 2, "fixed-length kernels take even M with at least two passes");
};

// Pass P of a radix order: butterfly j < MR = M / R reads entries j + q MR,
// multiplies entry q by w[k][q] (k = j mod Ns), transforms, and writes
// entry p to (j - k) R + k + p Ns.  A thread takes butterflies
// j = j0 + u JS, u < NU (the last sweep may be partial).
template <int M, int SH, int NT, bool REV, int P>
struct Pass {
    using G = Geo<M, SH, NT>;
    static constexpr RadixSeq S = REV ? G::REV : G::FWD;
    static constexpr int R = S.r[P], NS = S.ns[P], TOFF = S.toff[P];
    static constexpr int MR = M / R;
    static constexpr int NU = (MR + G::JS - 1) / G::JS;
    __device__ static bool live(int u, int j) { return MR % G::JS == 0 || u < NU - 1 || j < MR; }
    __device__ static int kof(int j0, int j) {
        if constexpr (NS == 1) return 0;
        else if constexpr (G::JS % NS == 0) return (int)((unsigned)j0 % NS);
        else return (int)((unsigned)j % NS);
    }
};

// Active length of a right-hand side, read without a branch (from this
// constant when the call has no per-right-hand-side lengths) so that the
// load can be issued early and waited for only where the length is used.
__device__ const int kNoLimit = 0x7fffffff;

__device__ __forceinline__ int active_raw(const SeriesIO& io, int outer) {
    typedef const __attribute__((address_space(1))) int gint;   // global memory: a plain vector load
    gint* p = io.nt_active ? (gint*)(io.nt_active + outer) : (gint*)&kNoLimit;
    return *p;
}
__device__ __forceinline__ int active_clamp(const SeriesIO& io, int raw) {
    return raw < 0 ? 0 : (raw < io.Nt ? raw : io.Nt);
}

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void apply_tw(cplx<T>* v, const cplx<T>* t) {
#pragma unroll
    for (int q = 1; q < R; ++q) v[q] = cmul(v[q], INV ? cconj(t[q - 1]) : t[q - 1]);
}

// Element at byte offset `off` from a workgroup-uniform base.  Bases advance
// by whole sweeps of bins or time steps (uniform arithmetic); the per-lane
// part is a 32-bit offset of fewer than JS bins or 2 JS time steps (the
// launchers check that it fits), so each access costs at most one address
// add instead of a 64-bit multiply-add.
template <typename E>
__device__ __forceinline__ E ld(const E* base, uint32_t off) {
    return *reinterpret_cast<const E*>(reinterpret_cast<const char*>(base) + off);
}
template <typename E>
__device__ __forceinline__ void st(E* base, uint32_t off, E v) {
    *reinterpret_cast<E*>(reinterpret_cast<char*>(base) + off) = v;
}

// ---------------------------------------------------------------- twiddle staging
// twg: e^{-2 pi i n / L}, n < L = 2M.  Pair table: W^k, k <= M / 2.  Pass
// table of a radix order: pass P's entry k (R - 1) + q - 1 is
// e^{-2 pi i q k / (Ns R)} = twg[q k L / (Ns R)].
template <typename T, int M, int SH, int NT>
__device__ __forceinline__ void stage_pair_tw(cplx<T>* twq, const cplx<T>* __restrict__ twg) {
    for (int k = threadIdx.x; k < Geo<M, SH, NT>::NPAIR; k += NT) twq[k] = twg[k];
}

template <typename T, int M, int SH, int NT, bool REV>
__device__ __forceinline__ void stage_pass_tw(cplx<T>* tab, const cplx<T>* __restrict__ twg) {
    static_for<0, Geo<M, SH, NT>::NP>([&](auto pc) {
        using Ps = Pass<M, SH, NT, REV, decltype(pc)::value>;
        constexpr int R = Ps::R, NS = Ps::NS, STEP = 2 * M / (NS * R);
        for (int e = threadIdx.x; e < NS * (R - 1); e += NT) {
            const int k = e / (R - 1), q = e - k * (R - 1) + 1;
            tab[Ps::TOFF + e] = twg[q * k * STEP];
        }
    });
}

// ---------------------------------------------------------------- passes
// Pass P on the LDS tile (read, barrier, write, barrier).
template <typename T, int M, int SH, int NT, bool REV, bool INV, int P>
__device__ __forceinline__ void lds_pass(cplx<T>* buf, const cplx<T>* tab, int s, int j0) {
    using Z = cplx<T>;
    using G = Geo<M, SH, NT>;
    using Ps = Pass<M, SH, NT, REV, P>;
    constexpr int R = Ps::R, NS = Ps::NS, MR = Ps::MR, NU = Ps::NU, RS = G::RS, JS = G::JS;
    Z v[NU][R];
    const Z* rb = buf + j0 * RS + s;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int j = j0 + u * JS;
        if (Ps::live(u, j)) {
#pragma unroll
            for (int q = 0; q < R; ++q) v[u][q] = rb[(u * JS + q * MR) * RS];
            if constexpr (NS > 1) apply_tw<T, R, INV>(v[u], tab + Ps::TOFF + Ps::kof(j0, j) * (R - 1));
            dft_small<T, R, INV>(v[u]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int j = j0 + u * JS;
        if (Ps::live(u, j)) {
            const int k = Ps::kof(j0, j);
            Z* wb = buf + (j * R - k * (R - 1)) * RS + s;
#pragma unroll
            for (int p = 0; p < R; ++p) wb[p * NS * RS] = v[u][p];
        }
    }
    __syncthreads();
}

// First forward pass fed by the time series (src: series s0 at t = 0; lane
// s reads series s0 + s): z[n] = x[2n] + i x[2n+1], x[t] = 0 for t >= nt or
// for a series past S (ok false).
template <typename T, typename TIN, int M, int SH, int NT>
__device__ __forceinline__ void first_pass_from_time(cplx<T>* buf, const TIN* __restrict__ src, long long t_stride,
                                                     bool ok, int nt, int s, int j0) {
    const uint32_t ts = (uint32_t)t_stride * (uint32_t)sizeof(TIN);
    uint32_t o0 = 2u * (uint32_t)j0 * ts + (uint32_t)s * (uint32_t)sizeof(TIN);   // t = 2 j0 from the sweep base
    asm volatile("" : "+v"(o0));
    using Z = cplx<T>;
    using G = Geo<M, SH, NT>;
    using Ps = Pass<M, SH, NT, false, 0>;
    constexpr int R = Ps::R, MR = Ps::MR, NU = Ps::NU, RS = G::RS, JS = G::JS;
    Z v[NU][R];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int j = j0 + u * JS;
        if (Ps::live(u, j)) {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int t0 = 2 * (j + q * MR);
                T x0 = T(0), x1 = T(0);
                const TIN* sb = src + (long long)(2 * (u * JS + q * MR)) * t_stride;   // t = 2 (u JS + q MR)
                if (ok && t0 < nt) x0 = (T)ld(sb, o0);
                if (ok && t0 + 1 < nt) x1 = (T)ld(sb, o0 + ts);
                v[u][q] = cmk<T>(x0, x1);
            }
            dft_small<T, R, false>(v[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int j = j0 + u * JS;
        if (Ps::live(u, j)) {
            Z* wb = buf + j * R * RS + s;
#pragma unroll
            for (int p = 0; p < R; ++p) wb[p * RS] = v[u][p];
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- real <-> half spectrum, by bin pairs
// Inverse pre-step: Z[k] = E + i O with E = (X[k] + conj X[M-k]) / 2,
// O = conj(W^k) (X[k] - conj X[M-k]) / 2.
template <typename T>
__device__ __forceinline__ cplx<T> pre_one(cplx<T> xa, cplx<T> xb, cplx<T> w) {
    const cplx<T> cb = cconj(xb);
    const cplx<T> e = cadd(xa, cb);
    const cplx<T> o = cmul(cconj(w), csub(xa, cb));
    return cmk<T>(T(0.5) * (e.x - o.y), T(0.5) * (e.y + o.x));
}

// Forward post-step: X[k] = (Z[k] + conj Z[M-k]) / 2 - (i/2) W^k (Z[k] - conj Z[M-k]).
template <typename T>
__device__ __forceinline__ cplx<T> post_one(cplx<T> a, cplx<T> b, cplx<T> w) {
    const cplx<T> cb = cconj(b);
    const cplx<T> sum = cadd(a, cb);
    const cplx<T> t = cmul(w, csub(a, cb));
    return cmk<T>(T(0.5) * (sum.x + t.y), T(0.5) * (sum.y - t.x));
}

// Half spectra X[0..M] (sum of nparts partials; zero for a series past S)
// into Z[0..M-1] on the tile.  Bins 0 and M are taken as real.  src: series
// s0 of bin 0 of partial 0; lane s reads series s0 + s.
template <typename T, int M, int SH, int NT>
__device__ __forceinline__ void load_pre(cplx<T>* buf, const cplx<T>* twq, const cplx<T>* __restrict__ src,
                                         const SeriesIO& io, bool ok, int s, int j0) {
    using Z = cplx<T>;
    using G = Geo<M, SH, NT>;
    constexpr int RS = G::RS, JS = G::JS, NU = (G::NPAIR + JS - 1) / JS;
    // bin k = j0 + u JS: base row u JS, lane offset j0 rows; bin M - k: base
    // row M - (JS - 1) - u JS, lane offset JS - 1 - j0 rows
    static_assert(M - (JS - 1) - (NU - 1) * JS >= 0, "partner rows start inside the spectrum");
    const uint32_t fs = (uint32_t)io.f_stride * (uint32_t)sizeof(Z), so = (uint32_t)s * (uint32_t)sizeof(Z);
    const uint32_t oa = (uint32_t)j0 * fs + so, ob = (uint32_t)(JS - 1 - j0) * fs + so;
    Z xa[NU], xb[NU];
    auto gather = [&](const Z* sp, Z (&va)[NU], Z (&vb)[NU]) {
        // opaque copies: keeps each offset computation next to its load, where
        // it is matched as a 32-bit offset from a scalar base
        uint32_t a0 = oa, b0 = ob;
        asm volatile("" : "+v"(a0), "+v"(b0));
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            if (u < NU - 1 || j0 + u * JS < G::NPAIR) {
                va[u] = ld(sp + (long long)(u * JS) * io.f_stride, a0);
                vb[u] = ld(sp + (long long)(M - (JS - 1) - u * JS) * io.f_stride, b0);
            }
        }
    };
    if (ok) {
        gather(src, xa, xb);
        for (int part = 1; part < io.nparts; ++part) {
            Z va[NU], vb[NU];
            gather(src + (long long)part * io.f_part, va, vb);
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                if (u < NU - 1 || j0 + u * JS < G::NPAIR) {
                    xa[u] = cadd(xa[u], va[u]);
                    xb[u] = cadd(xb[u], vb[u]);
                }
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < NU; ++u) xa[u] = xb[u] = cmk<T>(T(0), T(0));
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int k = j0 + u * JS;
        if (u < NU - 1 || k < G::NPAIR) {
            Z a = xa[u], b = xb[u];
            if (u == 0 && k == 0) { a.y = T(0); b.y = T(0); }
            const Z w = twq[k];
            buf[k * RS + s] = pre_one<T>(a, b, w);
            if ((u > 0 || k > 0) && 2 * k != M) buf[(M - k) * RS + s] = pre_one<T>(b, a, cmk<T>(-w.x, w.y));
        }
    }
    __syncthreads();
}

// Half spectra X[0..M] from Z[0..M-1] on the tile, to row[k f_stride + s0 + s]
// (complex, or quad BF16 hi/lo for FP32 with io.quad) for series below S_pad.
// With STAGED, quad output goes through LDS (over the tile, after a
// barrier): each lane first packs its bins' hi/lo words into the tile's bin
// rows of 8 TW bytes in storage order, then the workgroup stores them 16
// bytes per lane, a quarter of the store instructions of per-word stores
// (measured: r2c at 64 RHS 8 % faster; the re-pad, whose time is its
// arithmetic, 1 % slower, so it stores per word).
// With amax_slot (FP32 complex output only), each wavefront's largest |re|,
// |im| of the values it stores goes to amax_slot[wavefront].
template <typename T, int M, int SH, int NT, bool STAGED>
__device__ __forceinline__ void post_store(cplx<T>* buf, const cplx<T>* twq, const SeriesIO& io, cplx<T>* row,
                                           int s0, int s, int j0, float* amax_slot) {
    using Z = cplx<T>;
    using G = Geo<M, SH, NT>;
    constexpr int RS = G::RS, JS = G::JS, NU = (G::NPAIR + JS - 1) / JS;
    if constexpr (sizeof(T) == sizeof(float) && STAGED) {
        if (io.quad) {
            constexpr int TW = G::TW, RB = 8 * TW;        // staged bytes per bin row
            static_assert(TW % 4 == 0 && (M + 1) * RB <= G::TILE * (int)sizeof(Z), "staged rows fit the tile");
            uint32_t hk[NU][2], hm[NU][2];                // (hi, lo) of bins k and M - k
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int k = j0 + u * JS;
                if (u < NU - 1 || k < G::NPAIR) {
                    const int km = (u == 0 && k == 0) ? 0 : M - k;
                    const Z a = buf[k * RS + s], b = buf[km * RS + s];
                    const Z w = twq[k];
                    const Z xk = post_one<T>(a, b, w);
                    const Z xm = post_one<T>(b, a, cmk<T>(-w.x, w.y));
                    hk[u][0] = pack_bf16_rne(xk.x, xk.y);
                    hk[u][1] = pack_bf16_rne(xk.x - __uint_as_float(hk[u][0] << 16),
                                             xk.y - __uint_as_float(hk[u][0] & 0xffff0000u));
                    hm[u][0] = pack_bf16_rne(xm.x, xm.y);
                    hm[u][1] = pack_bf16_rne(xm.x - __uint_as_float(hm[u][0] << 16),
                                             xm.y - __uint_as_float(hm[u][0] & 0xffff0000u));
                }
            }
            __syncthreads();                              // every lane is done reading the tile
            uint32_t* sg = reinterpret_cast<uint32_t*>(buf);
            const int wo = 8 * (s >> 2) + (s & 3);        // word of series s in its bin row (hi; lo 4 further)
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int k = j0 + u * JS;
                if (u < NU - 1 || k < G::NPAIR) {
                    sg[k * (RB / 4) + wo] = hk[u][0];
                    sg[k * (RB / 4) + wo + 4] = hk[u][1];
                    if (2 * k != M) {
                        const int km = (u == 0 && k == 0) ? M : M - k;
                        sg[km * (RB / 4) + wo] = hm[u][0];
                        sg[km * (RB / 4) + wo + 4] = hm[u][1];
                    }
                }
            }
            __syncthreads();
            // 16-byte chunk c of bin b: series 4 (c / 2) .. + 3, hi (even c) or lo
            constexpr int CPB = RB / 16;                  // chunks per bin row
            uint8_t* const out = reinterpret_cast<uint8_t*>(row + s0);
            const long long fsb = (long long)io.f_stride * (long long)sizeof(Z);
            for (int e = threadIdx.x; e < (M + 1) * CPB; e += NT) {
                const int bin = e / CPB, c = e % CPB;
                if (s0 + 4 * (c >> 1) < io.S_pad)
                    *reinterpret_cast<uint4*>(out + bin * fsb + c * 16) =
                        *reinterpret_cast<const uint4*>(reinterpret_cast<const uint8_t*>(sg) + bin * RB + c * 16);
            }
            return;
        }
    }
    const bool ok = s0 + s < io.S_pad;
    // quad storage: series c of a bin is word 8 (c / 4) + c % 4 (hi) and 4 words
    // further (lo) from the bin's first word; tiles start at multiples of 4
    bool quad = false;
    if constexpr (sizeof(T) == sizeof(float)) quad = io.quad != 0;
    static_assert(M - (JS - 1) - (NU - 1) * JS >= 0, "partner rows start inside the spectrum");
    Z* const rb = row + s0;
    const uint32_t fs = (uint32_t)io.f_stride * (uint32_t)sizeof(Z);
    const uint32_t lo_ = quad ? (uint32_t)(8 * (s >> 2) + (s & 3)) * 4u : (uint32_t)s * (uint32_t)sizeof(Z);
    // bins k = j0 + u JS and M - k from base rows u JS and M - (JS - 1) - u JS
    uint32_t oa = (uint32_t)j0 * fs + lo_, ob = (uint32_t)(JS - 1 - j0) * fs + lo_;
    asm volatile("" : "+v"(oa), "+v"(ob));
    float vmax = 0.f;
    auto put = [&](Z* rbase, uint32_t off, Z X) {
        if constexpr (sizeof(T) == sizeof(float)) {
            vmax = fmaxf(vmax, fmaxf(fabsf(X.x), fabsf(X.y)));
            if (quad) {
                const uint32_t hi = pack_bf16_rne(X.x, X.y);
                const uint32_t lo = pack_bf16_rne(X.x - __uint_as_float(hi << 16), X.y - __uint_as_float(hi & 0xffff0000u));
                uint32_t* qb = reinterpret_cast<uint32_t*>(rbase);
                st(qb, off, hi);
                st(qb, off + 16u, lo);
                return;
            }
        }
        st(rbase, off, X);
    };
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int k = j0 + u * JS;
        if (u < NU - 1 || k < G::NPAIR) {
            const int km = (u == 0 && k == 0) ? 0 : M - k;     // Z is M-periodic
            const Z a = buf[k * RS + s], b = buf[km * RS + s];
            const Z w = twq[k];
            const Z xk = post_one<T>(a, b, w);
            const Z xm = post_one<T>(b, a, cmk<T>(-w.x, w.y));
            if (ok) {
                put(rb + (long long)(u * JS) * io.f_stride, oa, xk);
                if (2 * k != M) put(rb + (long long)(M - (JS - 1) - u * JS) * io.f_stride, ob, xm);
            }
        }
    }
    if constexpr (sizeof(T) == sizeof(float)) {
        if (amax_slot) wave_amax_store(vmax, amax_slot);
    }
}

// Slots of this tile's wavefront maxima (one per wavefront of an NT-thread
// workgroup), or nullptr.
template <int NT>
__device__ __forceinline__ float* amax_slots_of(const SeriesIO& io, int outer, int tile) {
    return io.amax_part ? io.amax_part + (long long)outer * io.amax_slots + tile * (NT / 64) : nullptr;
}

// The re-pad's merged pass on one butterfly (after its inverse twiddles):
// inverse radix-R DFT to z[j + p MR], p < R; keep the time values of the
// active length (t = 2n, 2n + 1 < nt) scaled by 1 / M; forward radix-R DFT
// of the result.  With R = 4 the outputs p = 2, 3 are time indices
// n >= 2 MR = M / 2, i.e. t >= M >= Nt >= nt (M = L / 2 is at least Nt), so
// they are zero for every active length: the inverse forms outputs 0 and 1
// only (12 additions instead of 16) and the forward takes (z0, z1, 0, 0)
// (8 instead of 16); other radices take the general form.
template <typename T, int R, int MR>
__device__ __forceinline__ void truncate_repad_pass(cplx<T>* a, int j, int nt, T inv) {
    using Z = cplx<T>;
    if constexpr (R == 4) {
        const Z t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
        const Z t2 = cadd(a[1], a[3]), t3 = csub(a[1], a[3]);
        Z z0 = cadd(t0, t2);
        Z z1 = cmk<T>(t1.x - t3.y, t1.y + t3.x);              // t1 + i t3
        const int n0 = j, n1 = j + MR;
        z0.x = (2 * n0 < nt) ? z0.x * inv : T(0);
        z0.y = (2 * n0 + 1 < nt) ? z0.y * inv : T(0);
        z1.x = (2 * n1 < nt) ? z1.x * inv : T(0);
        z1.y = (2 * n1 + 1 < nt) ? z1.y * inv : T(0);
        a[0] = cadd(z0, z1);
        a[2] = csub(z0, z1);
        a[1] = cmk<T>(z0.x + z1.y, z0.y - z1.x);               // z0 - i z1
        a[3] = cmk<T>(z0.x - z1.y, z0.y + z1.x);               // z0 + i z1
    } else {
        dft_small<T, R, true>(a);
#pragma unroll
        for (int p = 0; p < R; ++p) {
            const int n = j + p * MR;
            a[p].x = (2 * n < nt) ? a[p].x * inv : T(0);
            a[p].y = (2 * n + 1 < nt) ? a[p].y * inv : T(0);
        }
        dft_small<T, R, false>(a);
    }
}

// ---------------------------------------------------------------- kernels
// Persistent item loop: workgroup b runs on XCD b % 8 and takes the items
// x Q + i, i = b / 8, b / 8 + G / 8, ... of that XCD's share [x Q, (x + 1) Q)
// (G = grid size, a multiple of 8): at any time the workgroups of one XCD
// work on adjacent tiles.
template <typename T, typename TIN, int M, int SH, int NT>
__global__ __launch_bounds__(NT) void k_r2c_fx(SeriesIO io, const TIN* __restrict__ in,
                                                       cplx<T>* __restrict__ out, const cplx<T>* __restrict__ twg,
                                                       ItemMap im) {
    using Z = cplx<T>;
    using G = Geo<M, SH, NT>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Z* buf = reinterpret_cast<Z*>(smem_raw);
    Z* twq = buf + G::TILE;
    Z* twf = twq + G::NPAIR;
    stage_pair_tw<T, M, SH, NT>(twq, twg);
    stage_pass_tw<T, M, SH, NT, false>(twf, twg);
    __syncthreads();
    const int s_ = threadIdx.x & (G::TW - 1), j0_ = threadIdx.x >> SH;
    const int xq = (int)(blockIdx.x & 7) * im.Q, nper = (int)(gridDim.x >> 3);
    for (int i = (int)(blockIdx.x >> 3); i < im.Q && xq + i < im.items; i += nper) {
        const int outer = (xq + i) / im.ntiles, tile = xq + i - outer * im.ntiles;
        // Fresh copies of the lane indices each tile: otherwise every address
        // derived from them is hoisted out of the loop and held in registers.
        int s = s_, j0 = j0_;
        asm volatile("" : "+v"(s), "+v"(j0));
        const int s0 = tile << SH;
        const int nt = active_clamp(io, active_raw(io, outer));
        first_pass_from_time<T, TIN, M, SH, NT>(buf, in + (long long)outer * io.t_outer + s0, io.t_stride,
                                            s0 + s < io.S, nt, s, j0);
        static_for<1, G::NP>([&](auto pc) { lds_pass<T, M, SH, NT, false, false, decltype(pc)::value>(buf, twf, s, j0); });
        post_store<T, M, SH, NT, true>(buf, twq, io, out + (long long)outer * io.f_outer, s0, s, j0,
                                   amax_slots_of<NT>(io, outer, tile));
        __syncthreads();
    }
}

template <typename T, typename TOUT, int M, int SH, int NT, int EPI>
__global__ __launch_bounds__(NT) void k_c2r_fx(SeriesIO io, const cplx<T>* __restrict__ in,
                                                       TOUT* __restrict__ out, const cplx<T>* __restrict__ twg,
                                                       MisfitArgs ma, ItemMap im) {
    using Z = cplx<T>;
    using G = Geo<M, SH, NT>;
    using Pl = Pass<M, SH, NT, true, G::NP - 1>;
    constexpr int R = Pl::R, NS = Pl::NS, MR = Pl::MR, NU = Pl::NU, RS = G::RS, JS = G::JS;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Z* buf = reinterpret_cast<Z*>(smem_raw);
    Z* twq = buf + G::TILE;
    Z* twr = twq + G::NPAIR;
    stage_pair_tw<T, M, SH, NT>(twq, twg);
    stage_pass_tw<T, M, SH, NT, true>(twr, twg);
    __syncthreads();
    const int s_ = threadIdx.x & (G::TW - 1), j0_ = threadIdx.x >> SH;
    const T inv = T(1) / T(M);
    const int xq = (int)(blockIdx.x & 7) * im.Q, nper = (int)(gridDim.x >> 3);
    for (int i = (int)(blockIdx.x >> 3); i < im.Q && xq + i < im.items; i += nper) {
        const int outer = (xq + i) / im.ntiles, tile = xq + i - outer * im.ntiles;
        // Fresh copies of the lane indices each tile: otherwise every address
        // derived from them is hoisted out of the loop and held in registers.
        int s = s_, j0 = j0_;
        asm volatile("" : "+v"(s), "+v"(j0));
        const int s0 = tile << SH;
        const int col = s0 + s;
        const bool ok = col < io.S;
        const int nt_raw = active_raw(io, outer);      // used after the transform
        load_pre<T, M, SH, NT>(buf, twq, in + (long long)outer * io.f_outer + s0, io, ok, s, j0);
        const int nt = active_clamp(io, nt_raw);
        static_for<0, G::NP - 1>([&](auto pc) { lds_pass<T, M, SH, NT, true, true, decltype(pc)::value>(buf, twr, s, j0); });
        // last inverse pass: butterfly j (< MR = NS) writes z[j + p NS] straight to the time series
        Z v[NU][R];
        const Z* rb = buf + j0 * RS + s;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int j = j0 + u * JS;
            if (Pl::live(u, j)) {
#pragma unroll
                for (int q = 0; q < R; ++q) v[u][q] = rb[(u * JS + q * MR) * RS];
                apply_tw<T, R, true>(v[u], twr + Pl::TOFF + j * (R - 1));
                dft_small<T, R, true>(v[u]);
            }
        }
        TOUT* dst = out + (long long)outer * io.t_outer + s0;
        const uint32_t ts = (uint32_t)io.t_stride * (uint32_t)sizeof(TOUT);
        uint32_t o0 = 2u * (uint32_t)j0 * ts + (uint32_t)s * (uint32_t)sizeof(TOUT);   // t = 2 j0
        asm volatile("" : "+v"(o0));
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int j = j0 + u * JS;
            if (ok && Pl::live(u, j)) {
#pragma unroll
                for (int p = 0; p < R; ++p) {
                    const int n = j + p * NS;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int t = 2 * n + h;
                        if (t < io.Nt) {
                            const T y = (h == 0 ? v[u][p].x : v[u][p].y) * inv;
                            const long long trow = 2 * (u * JS + p * NS) + h;   // t - 2 j0
                            const uint32_t off = o0;
                            if constexpr (EPI == EPI_PLAIN) {
                                st(dst + trow * io.t_stride, off, (t < nt) ? (TOUT)y : TOUT(0));
                            } else {
                                const TOUT* dob = reinterpret_cast<const TOUT*>(ma.d_obs) + (long long)outer * io.t_outer + s0;
                                double wv = 0.0;
                                if (t < nt) {
                                    const double var = ma.var_mode == 0 ? ma.var[0]
                                                     : ma.var_mode == 1 ? ma.var[col]
                                                                        : ma.var[(long long)t * io.S + col];
                                    const double r = (double)y - (double)ld(dob + trow * io.t_stride, off);
                                    wv = r / var;
                                    acc += r * wv;
                                }
                                st(dst + trow * io.t_stride, off, (TOUT)wv);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();                       // tile reads done: the LDS is free
        if constexpr (EPI == EPI_MISFIT) {
            static_assert(G::TILE * sizeof(Z) >= NT * sizeof(double), "reduction fits in the tile");
            double* red = reinterpret_cast<double*>(smem_raw);
            red[threadIdx.x] = acc;
            __syncthreads();
            for (int w = NT / 2; w > 0; w >>= 1) {
                if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
                __syncthreads();
            }
            if (threadIdx.x == 0) ma.partials[(long long)outer * im.ntiles + tile] = red[0];
            __syncthreads();
        }
    }
}

// Truncate-and-repad (see k_project in fft.hip), written over partial 0.
template <typename T, int M, int SH, int NT>
__global__ __launch_bounds__(NT) void k_project_fx(SeriesIO io, cplx<T>* in_out,
                                                           const cplx<T>* __restrict__ twg, ItemMap im) {
    using Z = cplx<T>;
    using G = Geo<M, SH, NT>;
    using Pl = Pass<M, SH, NT, true, G::NP - 1>;    // last inverse pass
    using Pf = Pass<M, SH, NT, false, 0>;           // first forward pass: same radix, same index sets
    static_assert(Pl::R == Pf::R && Pl::NS == Pf::MR, "reversed order ends with the forward order's first radix");
    constexpr int R = Pl::R, MR = Pl::MR, NU = Pl::NU, RS = G::RS, JS = G::JS;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Z* buf = reinterpret_cast<Z*>(smem_raw);
    Z* twq = buf + G::TILE;
    Z* twf = twq + G::NPAIR;
    Z* twr = twf + (M - 1);
    stage_pair_tw<T, M, SH, NT>(twq, twg);
    stage_pass_tw<T, M, SH, NT, false>(twf, twg);
    stage_pass_tw<T, M, SH, NT, true>(twr, twg);
    __syncthreads();
    const int s_ = threadIdx.x & (G::TW - 1), j0_ = threadIdx.x >> SH;
    const T inv = T(1) / T(M);
    const int xq = (int)(blockIdx.x & 7) * im.Q, nper = (int)(gridDim.x >> 3);
    for (int i = (int)(blockIdx.x >> 3); i < im.Q && xq + i < im.items; i += nper) {
        const int outer = (xq + i) / im.ntiles, tile = xq + i - outer * im.ntiles;
        // Fresh copies of the lane indices each tile: otherwise every address
        // derived from them is hoisted out of the loop and held in registers.
        int s = s_, j0 = j0_;
        asm volatile("" : "+v"(s), "+v"(j0));
        const int s0 = tile << SH;
        const int nt_raw = active_raw(io, outer);      // used between the transforms
        Z* base = in_out + (long long)outer * io.f_outer;
        load_pre<T, M, SH, NT>(buf, twq, base + s0, io, s0 + s < io.S, s, j0);
        const int nt = active_clamp(io, nt_raw);
        static_for<0, G::NP - 1>([&](auto pc) { lds_pass<T, M, SH, NT, true, true, decltype(pc)::value>(buf, twr, s, j0); });
        // last inverse pass -> z[j + p MR]; keep t < nt (t = 2n, 2n + 1) and
        // scale by 1 / M; first forward pass on the same entries
        Z v[NU][R];
        const Z* rb = buf + j0 * RS + s;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int j = j0 + u * JS;
            if (Pl::live(u, j)) {
#pragma unroll
                for (int q = 0; q < R; ++q) v[u][q] = rb[(u * JS + q * MR) * RS];
                apply_tw<T, R, true>(v[u], twr + Pl::TOFF + j * (R - 1));
                truncate_repad_pass<T, R, MR>(v[u], j, nt, inv);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int j = j0 + u * JS;
            if (Pl::live(u, j)) {
                Z* wb = buf + j * R * RS + s;
#pragma unroll
                for (int p = 0; p < R; ++p) wb[p * RS] = v[u][p];
            }
        }
        __syncthreads();
        static_for<1, G::NP>([&](auto pc) { lds_pass<T, M, SH, NT, false, false, decltype(pc)::value>(buf, twf, s, j0); });
        post_store<T, M, SH, NT, false>(buf, twq, io, base, s0, s, j0, amax_slots_of<NT>(io, outer, tile));
        __syncthreads();
    }
}

// ---------------------------------------------------------------- FP16 operands of data-space columns
// Truncate-and-repad on FP16 (re, im) pairs, in place: the adjoint products
// arrive multiplied by sx[outer] and leave, re-padded, multiplied by
// sy[outer] (the forward products' FP16 right-hand sides).  One partial sum;
// the same transform as k_project_fx in FP32 between the conversions.
__device__ __forceinline__ float2 f16pair(uint32_t w, float s) { return make_float2(f16lo(w) * s, f16hi(w) * s); }
__device__ __forceinline__ uint32_t pair_f16(float re, float im, float s) {
    return f32_to_f16_rne(re * s) | (f32_to_f16_rne(im * s) << 16);
}

template <int M, int SH, int NT>
__device__ __forceinline__ void load_pre_h(float2* buf, const float2* twq, const uint32_t* __restrict__ src,
                                           const SeriesIO& io, bool ok, int s, int j0, float inv) {
    using Z = float2;
    using G = Geo<M, SH, NT>;
    constexpr int RS = G::RS, JS = G::JS, NU = (G::NPAIR + JS - 1) / JS;
    static_assert(M - (JS - 1) - (NU - 1) * JS >= 0, "partner rows start inside the spectrum");
    const uint32_t fs = (uint32_t)io.f_stride * 4u, so = (uint32_t)s * 4u;
    uint32_t a0 = (uint32_t)j0 * fs + so, b0 = (uint32_t)(JS - 1 - j0) * fs + so;
    asm volatile("" : "+v"(a0), "+v"(b0));
    Z xa[NU], xb[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        if (u < NU - 1 || j0 + u * JS < G::NPAIR) {
            if (ok) {
                xa[u] = f16pair(ld(src + (long long)(u * JS) * io.f_stride, a0), inv);
                xb[u] = f16pair(ld(src + (long long)(M - (JS - 1) - u * JS) * io.f_stride, b0), inv);
            } else {
                xa[u] = xb[u] = cmk<float>(0.f, 0.f);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int k = j0 + u * JS;
        if (u < NU - 1 || k < G::NPAIR) {
            Z a = xa[u], b = xb[u];
            if (u == 0 && k == 0) { a.y = 0.f; b.y = 0.f; }
            const Z w = twq[k];
            buf[k * RS + s] = pre_one<float>(a, b, w);
            if ((u > 0 || k > 0) && 2 * k != M) buf[(M - k) * RS + s] = pre_one<float>(b, a, cmk<float>(-w.x, w.y));
        }
    }
    __syncthreads();
}

template <int M, int SH, int NT>
__device__ __forceinline__ void post_store_h(float2* buf, const float2* twq, const SeriesIO& io, uint32_t* row, int s0,
                                             int s, int j0, float sc) {
    using Z = float2;
    using G = Geo<M, SH, NT>;
    constexpr int RS = G::RS, JS = G::JS, NU = (G::NPAIR + JS - 1) / JS;
    static_assert(M - (JS - 1) - (NU - 1) * JS >= 0, "partner rows start inside the spectrum");
    const bool ok = s0 + s < io.S_pad;
    uint32_t* const rb = row + s0;
    const uint32_t fs = (uint32_t)io.f_stride * 4u, lo_ = (uint32_t)s * 4u;
    uint32_t oa = (uint32_t)j0 * fs + lo_, ob = (uint32_t)(JS - 1 - j0) * fs + lo_;
    asm volatile("" : "+v"(oa), "+v"(ob));
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int k = j0 + u * JS;
        if (u < NU - 1 || k < G::NPAIR) {
            const int km = (u == 0 && k == 0) ? 0 : M - k;
            const Z a = buf[k * RS + s], b = buf[km * RS + s];
            const Z w = twq[k];
            const Z xk = post_one<float>(a, b, w);
            const Z xm = post_one<float>(b, a, cmk<float>(-w.x, w.y));
            if (ok) {
                st(rb + (long long)(u * JS) * io.f_stride, oa, pair_f16(xk.x, xk.y, sc));
                if (2 * k != M) st(rb + (long long)(M - (JS - 1) - u * JS) * io.f_stride, ob, pair_f16(xm.x, xm.y, sc));
            }
        }
    }
}

template <int M, int SH, int NT>
__global__ __launch_bounds__(NT) void k_project_fx_h(SeriesIO io, uint32_t* in_out,
                                                             const float2* __restrict__ twg, const float* __restrict__ sx,
                                                             const float* __restrict__ sy, ItemMap im) {
    using T = float;
    using Z = float2;
    using G = Geo<M, SH, NT>;
    using Pl = Pass<M, SH, NT, true, G::NP - 1>;
    using Pf = Pass<M, SH, NT, false, 0>;
    static_assert(Pl::R == Pf::R && Pl::NS == Pf::MR, "reversed order ends with the forward order's first radix");
    constexpr int R = Pl::R, MR = Pl::MR, NU = Pl::NU, RS = G::RS, JS = G::JS;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Z* buf = reinterpret_cast<Z*>(smem_raw);
    Z* twq = buf + G::TILE;
    Z* twf = twq + G::NPAIR;
    Z* twr = twf + (M - 1);
    stage_pair_tw<T, M, SH, NT>(twq, twg);
    stage_pass_tw<T, M, SH, NT, false>(twf, twg);
    stage_pass_tw<T, M, SH, NT, true>(twr, twg);
    __syncthreads();
    const int s_ = threadIdx.x & (G::TW - 1), j0_ = threadIdx.x >> SH;
    const T inv = T(1) / T(M);
    const int xq = (int)(blockIdx.x & 7) * im.Q, nper = (int)(gridDim.x >> 3);
    for (int i = (int)(blockIdx.x >> 3); i < im.Q && xq + i < im.items; i += nper) {
        const int outer = (xq + i) / im.ntiles, tile = xq + i - outer * im.ntiles;
        int s = s_, j0 = j0_;
        asm volatile("" : "+v"(s), "+v"(j0));
        const int s0 = tile << SH;
        const int nt_raw = active_raw(io, outer);
        uint32_t* base = in_out + (long long)outer * io.f_outer;
        load_pre_h<M, SH, NT>(buf, twq, base + s0, io, s0 + s < io.S, s, j0, 1.f / sx[outer]);
        const int nt = active_clamp(io, nt_raw);
        static_for<0, G::NP - 1>([&](auto pc) { lds_pass<T, M, SH, NT, true, true, decltype(pc)::value>(buf, twr, s, j0); });
        Z v[NU][R];
        const Z* rbp = buf + j0 * RS + s;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int j = j0 + u * JS;
            if (Pl::live(u, j)) {
#pragma unroll
                for (int q = 0; q < R; ++q) v[u][q] = rbp[(u * JS + q * MR) * RS];
                apply_tw<T, R, true>(v[u], twr + Pl::TOFF + j * (R - 1));
                truncate_repad_pass<T, R, MR>(v[u], j, nt, inv);
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int j = j0 + u * JS;
            if (Pl::live(u, j)) {
                Z* wb = buf + j * R * RS + s;
#pragma unroll
                for (int p = 0; p < R; ++p) wb[p * RS] = v[u][p];
            }
        }
        __syncthreads();
        static_for<1, G::NP>([&](auto pc) { lds_pass<T, M, SH, NT, false, false, decltype(pc)::value>(buf, twf, s, j0); });
        post_store_h<M, SH, NT>(buf, twq, io, base, s0, s, j0, sy[outer]);
        __syncthreads();
    }
}

// ---------------------------------------------------------------- host side
template <int M, int SH, int NT>
constexpr size_t fx_lds(size_t zbytes, int ntables) {
    return ((size_t)Geo<M, SH, NT>::TILE + Geo<M, SH, NT>::NPAIR + (size_t)ntables * (M - 1)) * zbytes;
}

// Grid of resident workgroups for kernel K (occupancy per CU cached per
// kernel; the CU count is queried each time), at most 8 Q.
template <auto K, int NT>
dim3 fx_grid(size_t lds, const ItemMap& im) {
    static int occ = 0;
    if (occ == 0) {
        int o = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, K, NT, lds) != hipSuccess || o < 1) o = 1;
        occ = o;
    }
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        ncu = 256;
    const int per_xcd = (occ * ncu + 7) / 8;
    return dim3(8 * (unsigned)std::max(1, std::min(im.Q, per_xcd)));
}

ItemMap fx_items(int S, int sh, int outer) {
    ItemMap im;
    im.ntiles = (S + (1 << sh) - 1) >> sh;
    im.items = im.ntiles * outer;
    im.Q = (im.items + 7) / 8;
    return im;
}

template <typename T, int M, int SH, int NT>
hipError_t fx_r2c(bool in_f64, const SeriesIO& io, const void* in, void* out, const void* tw, hipStream_t st) {
    const ItemMap im = fx_items(io.S_pad, SH, io.outer_count);
    if (im.items == 0) return hipSuccess;
    if (io.amax_part && (long long)im.ntiles * (NT / 64) > io.amax_slots) return hipErrorInvalidValue;
    const size_t lds = fx_lds<M, SH, NT>(sizeof(cplx<T>), 1);
    if (in_f64) {
        constexpr auto k = k_r2c_fx<T, double, M, SH, NT>;
        hipLaunchKernelGGL(k, (fx_grid<k, NT>(lds, im)), dim3(NT), lds, st, io, (const double*)in, (cplx<T>*)out,
                           (const cplx<T>*)tw, im);
    } else {
        constexpr auto k = k_r2c_fx<T, float, M, SH, NT>;
        hipLaunchKernelGGL(k, (fx_grid<k, NT>(lds, im)), dim3(NT), lds, st, io, (const float*)in, (cplx<T>*)out,
                           (const cplx<T>*)tw, im);
    }
    return hipGetLastError();
}

template <typename T, int M, int SH, int NT>
hipError_t fx_c2r(const SeriesIO& io, const void* in, void* out, const void* tw, const MisfitArgs& ma,
                  hipStream_t st) {
    const ItemMap im = fx_items(io.S, SH, io.outer_count);
    if (im.items == 0) return hipSuccess;
    size_t lds = fx_lds<M, SH, NT>(sizeof(cplx<T>), 1);
    if (lds < NT * sizeof(double)) lds = NT * sizeof(double);
    if (ma.d_obs) {
        constexpr auto k = k_c2r_fx<T, T, M, SH, NT, EPI_MISFIT>;
        hipLaunchKernelGGL(k, (fx_grid<k, NT>(lds, im)), dim3(NT), lds, st, io, (const cplx<T>*)in, (T*)out,
                           (const cplx<T>*)tw, ma, im);
    } else {
        constexpr auto k = k_c2r_fx<T, T, M, SH, NT, EPI_PLAIN>;
        hipLaunchKernelGGL(k, (fx_grid<k, NT>(lds, im)), dim3(NT), lds, st, io, (const cplx<T>*)in, (T*)out,
                           (const cplx<T>*)tw, ma, im);
    }
    return hipGetLastError();
}

template <typename T, int M, int SH, int NT>
hipError_t fx_project(const SeriesIO& io, void* in_out, const void* tw, hipStream_t st) {
    const ItemMap im = fx_items(io.S_pad, SH, io.outer_count);
    if (im.items == 0) return hipSuccess;
    if (io.amax_part && (long long)im.ntiles * (NT / 64) > io.amax_slots) return hipErrorInvalidValue;
    if (io.Nt > M) return hipErrorInvalidValue;         // the merged pass drops time indices >= M
    const size_t lds = fx_lds<M, SH, NT>(sizeof(cplx<T>), 2);
    constexpr auto k = k_project_fx<T, M, SH, NT>;
    hipLaunchKernelGGL(k, (fx_grid<k, NT>(lds, im)), dim3(NT), lds, st, io, (cplx<T>*)in_out, (const cplx<T>*)tw, im);
    return hipGetLastError();
}

template <int M, int SH, int NT>
hipError_t fx_project_h(const SeriesIO& io, void* in_out, const void* tw, const float* sx, const float* sy,
                        hipStream_t st) {
    const ItemMap im = fx_items(io.S_pad, SH, io.outer_count);
    if (im.items == 0) return hipSuccess;
    if (io.Nt > M) return hipErrorInvalidValue;         // the merged pass drops time indices >= M
    const size_t lds = fx_lds<M, SH, NT>(sizeof(float2), 2);
    constexpr auto k = k_project_fx_h<M, SH, NT>;
    hipLaunchKernelGGL(k, (fx_grid<k, NT>(lds, im)), dim3(NT), lds, st, io, (uint32_t*)in_out, (const float2*)tw, sx, sy,
                       im);
    return hipGetLastError();
}

// Compiled (M, tile shift, workgroup size) cases: the transform lengths of
// the common workloads (Nt = 16, 128, 420, and 500 of section 5's problem),
// with the tile widths fft_tile_shift picks on 256-thread workgroups, plus
// wide FP32 tiles for transforms of many series (fixed_wide_shift): 16
// series per tile, so that each bin row of a complex FP32 tile is one whole
// 128-byte line (measured: stores of 64-byte rows run at 3.1 TB/s, of
// 128-byte rows at 5.4 TB/s), on 512-thread workgroups for M = 420 (the
// same work per thread as its 8-series tiles) and 256 for M = 500.
#define P2O_FX_CASES(X)      \
    X(float, 16, 5, 256)     \
    X(float, 128, 4, 256)    \
    X(float, 420, 3, 256)    \
    X(float, 420, 4, 512)    \
    X(float, 500, 2, 256)    \
    X(float, 500, 4, 256)    \
    X(double, 16, 5, 256)    \
    X(double, 128, 3, 256)   \
    X(double, 420, 2, 256)   \
    X(double, 500, 1, 256)

// The re-pad on FP16 pairs (data-space columns): the FP32 cases, with
// 512-thread workgroups on the 16-series tiles of M = 500 (at the paper's
// dimensions 56.8 -> 42.8 ms per 64-column call, where the FP32 re-pad ran
// 50.6 -> 106 ms with them: it keeps 256); M = 420 keeps 8-series tiles.
#define P2O_FX_CASES_H(X)    \
    X(float, 16, 5, 256)     \
    X(float, 128, 4, 256)    \
    X(float, 420, 3, 256)    \
    X(float, 500, 2, 256)    \
    X(float, 500, 4, 512)

// Lane offsets of `rows` rows of `stride` elements (plus a tile) fit the
// unsigned 32-bit byte offsets the kernels add to their bases (ld, st;
// rows: one sweep, NT >> shift bins or twice that many time steps).
bool fits32(long long rows, long long stride, size_t esz) {
    return (rows * stride + 64) * (long long)esz < (1LL << 32);
}

}  // namespace

// FP16 operands of data-space columns: the FP32 lengths with compiled
// kernels (the plan's tile shift for S_pad series); false if there is none.
bool launch_fixed_project_h(const FftPlan& pl, const SeriesIO& io, void* in_out, const void* tw, int sh,
                            const float* sx, const float* sy, hipStream_t st, hipError_t* err) {
    if (!pl.fixed || io.nparts != 1 || io.quad) return false;
#define X(T, M_, SH_, NT_)                                                             \
    if (sizeof(T) == 4 && pl.M == M_ && sh == SH_) {                                   \
        if (!fits32(NT_ >> SH_, io.f_stride, 4)) return false;                         \
        if (err) *err = fx_project_h<M_, SH_, NT_>(io, in_out, tw, sx, sy, st);        \
        return true;                                                                   \
    }
    P2O_FX_CASES_H(X)
#undef X
    return false;
}

int fixed_wide_shift(bool f64, const FftPlan& pl) { return !f64 && pl.fixed && (pl.M == 500 || pl.M == 420) ? 4 : -1; }

int fixed_tile_waves(bool f64, const FftPlan& pl, int sh) {
#define X(T, M_, SH_, NT_) \
    if ((sizeof(T) == 8) == f64 && pl.fixed && pl.M == M_ && sh == SH_) return NT_ / 64;
    P2O_FX_CASES(X)
#undef X
    return 4;
}

bool launch_fixed_r2c(bool f64, bool in_f64, const FftPlan& pl, const SeriesIO& io, const void* in, void* out,
                      const void* tw, int sh, hipStream_t st, hipError_t* err) {
    const size_t z = f64 ? 16 : 8;
    if (!pl.fixed) return false;
#define X(T, M_, SH_, NT_)                                                             \
    if ((sizeof(T) == 8) == f64 && pl.M == M_ && sh == SH_) {                          \
        constexpr int js = NT_ >> SH_;                                                 \
        if (!fits32(2 * js, io.t_stride, in_f64 ? 8 : 4) || !fits32(js, io.f_stride, z)) return false; \
        *err = fx_r2c<T, M_, SH_, NT_>(in_f64, io, in, out, tw, st);                   \
        return true;                                                                   \
    }
    P2O_FX_CASES(X)
#undef X
    return false;
}

bool launch_fixed_c2r(bool f64, const FftPlan& pl, const SeriesIO& io, const void* in, void* out, const void* tw,
                      int sh, const void* d_obs, const double* var, int var_mode, double* partials, hipStream_t st,
                      hipError_t* err) {
    const size_t z = f64 ? 16 : 8;
    if (!pl.fixed) return false;
    const MisfitArgs ma{d_obs, var, var_mode, partials};
#define X(T, M_, SH_, NT_)                                                             \
    if ((sizeof(T) == 8) == f64 && pl.M == M_ && sh == SH_) {                          \
        constexpr int js = NT_ >> SH_;                                                 \
        if (!fits32(2 * js, io.t_stride, z / 2) || !fits32(js, io.f_stride, z)) return false; \
        *err = fx_c2r<T, M_, SH_, NT_>(io, in, out, tw, ma, st);                       \
        return true;                                                                   \
    }
    P2O_FX_CASES(X)
#undef X
    return false;
}

bool launch_fixed_project(bool f64, const FftPlan& pl, const SeriesIO& io, void* in_out, const void* tw, int sh,
                          hipStream_t st, hipError_t* err) {
    if (!pl.fixed) return false;
#define X(T, M_, SH_, NT_)                                                             \
    if ((sizeof(T) == 8) == f64 && pl.M == M_ && sh == SH_) {                          \
        if (!fits32(NT_ >> SH_, io.f_stride, f64 ? 16 : 8)) return false;              \
        *err = fx_project<T, M_, SH_, NT_>(io, in_out, tw, st);                        \
        return true;                                                                   \
    }
    P2O_FX_CASES(X)
#undef X
    return false;
}

}  // namespace p2o
