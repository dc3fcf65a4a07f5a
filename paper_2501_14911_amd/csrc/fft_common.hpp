// Pieces shared by the runtime-length and the fixed-length FFT kernels:
// small DFT butterflies (radices 2, 3, 4, 5, 7, 8), the workgroup-to-tile
// map and the active length of a right-hand side.
#pragma once
#include "common.hpp"

namespace p2o {

// ---------------------------------------------------------------- butterflies
// cos(2 pi m / R) and sin(2 pi m / R), m = 1 .. (R - 1) / 2, for the odd
// prime radices (to 21 significant digits).
template <typename T, int R>
__device__ __forceinline__ constexpr T prime_cos(int m) {
    if constexpr (R == 3) return T(-0.5);
    if constexpr (R == 5) return m == 1 ? T(0.309016994374947424102) : T(-0.809016994374947424102);
    return m == 1 ? T(0.623489801858733530525) : m == 2 ? T(-0.222520933956314404289) : T(-0.900968867902419126236);
}
template <typename T, int R>
__device__ __forceinline__ constexpr T prime_sin(int m) {
    if constexpr (R == 3) return T(0.866025403784438646764);
    if constexpr (R == 5) return m == 1 ? T(0.951056516295153572116) : T(0.587785252292473129169);
    return m == 1 ? T(0.781831482468029808708) : m == 2 ? T(0.974927912181823607018) : T(0.433883739117558120476);
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_small(cplx<T>* a) {
    using Z = cplx<T>;
    if constexpr (R == 2) {
        Z t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    } else if constexpr (R == 4) {
        Z t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
        Z t2 = cadd(a[1], a[3]), t3 = csub(a[1], a[3]);
        a[0] = cadd(t0, t2);
        a[2] = csub(t0, t2);
        if constexpr (!INV) {   // multiply t3 by -i
            a[1] = cmk<T>(t1.x + t3.y, t1.y - t3.x);
            a[3] = cmk<T>(t1.x - t3.y, t1.y + t3.x);
        } else {                // multiply t3 by +i
            a[1] = cmk<T>(t1.x - t3.y, t1.y + t3.x);
            a[3] = cmk<T>(t1.x + t3.y, t1.y - t3.x);
        }
    } else if constexpr (R == 8) {
        Z e[4] = {a[0], a[2], a[4], a[6]};
        Z o[4] = {a[1], a[3], a[5], a[7]};
        dft_small<T, 4, INV>(e);
        dft_small<T, 4, INV>(o);
        const T c = T(0.70710678118654752440084436210485);   // sqrt(2)/2
        Z o1, o2, o3;
        if constexpr (!INV) {   // e^{-i pi p / 4} o_p
            o1 = cmk<T>(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
            o2 = cmk<T>(o[2].y, -o[2].x);
            o3 = cmk<T>(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
        } else {                // e^{+i pi p / 4} o_p
            o1 = cmk<T>(c * (o[1].x - o[1].y), c * (o[1].x + o[1].y));
            o2 = cmk<T>(-o[2].y, o[2].x);
            o3 = cmk<T>(-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y));
        }
        a[0] = cadd(e[0], o[0]); a[4] = csub(e[0], o[0]);
        a[1] = cadd(e[1], o1);   a[5] = csub(e[1], o1);
        a[2] = cadd(e[2], o2);   a[6] = csub(e[2], o2);
        a[3] = cadd(e[3], o3);   a[7] = csub(e[3], o3);
    } else {
        // odd prime radix.  With s_q = a_q + a_{R-q}, d_q = a_q - a_{R-q} and
        // theta = 2 pi p q / R, output p of the forward DFT is
        //   a_0 + sum_q s_q cos(theta) - i sum_q d_q sin(theta)
        // and output R - p the same with + i (q, p = 1 .. (R - 1) / 2): real
        // coefficients instead of complex roots, a third of the multiplies.
        constexpr int H = (R - 1) / 2;
        Z sm[H + 1], df[H + 1];
        Z a0 = a[0], out0 = a[0];
#pragma unroll
        for (int q = 1; q <= H; ++q) {
            sm[q] = cadd(a[q], a[R - q]);
            df[q] = csub(a[q], a[R - q]);
            out0 = cadd(out0, sm[q]);
        }
#pragma unroll
        for (int p = 1; p <= H; ++p) {
            T ar = a0.x, ai = a0.y, br = T(0), bi = T(0);
#pragma unroll
            for (int q = 1; q <= H; ++q) {
                const int m = (p * q) % R;
                const T c = prime_cos<T, R>(m <= H ? m : R - m);
                const T sn = m <= H ? prime_sin<T, R>(m) : -prime_sin<T, R>(R - m);
                ar += c * sm[q].x;
                ai += c * sm[q].y;
                br += sn * df[q].x;
                bi += sn * df[q].y;
            }
            if constexpr (!INV) {
                a[p] = cmk<T>(ar + bi, ai - br);
                a[R - p] = cmk<T>(ar - bi, ai + br);
            } else {
                a[p] = cmk<T>(ar - bi, ai + br);
                a[R - p] = cmk<T>(ar + bi, ai - br);
            }
        }
        a[0] = out0;
    }
}


// ---------------------------------------------------------------- work items
// Workgroup id -> (tile, outer) such that consecutive ids on one XCD (ids are
// dealt to the 8 XCDs round-robin) take adjacent column tiles and share L2 lines.
struct ItemMap {
    int ntiles;   // column tiles per outer index
    int items;    // ntiles * outer count
    int Q;        // ceil(items / 8)
};

__device__ __forceinline__ bool fft_item(const ItemMap& im, int& tile, int& outer) {
    const int q = (int)(blockIdx.x & 7) * im.Q + (int)(blockIdx.x >> 3);
    if (q >= im.items) return false;
    outer = q / im.ntiles;
    tile = q - outer * im.ntiles;
    return true;
}

__device__ __forceinline__ int active_len(const SeriesIO& io, int outer) {
    int nt = io.Nt;
    if (io.nt_active) {
        const int a = io.nt_active[outer];
        nt = a < 0 ? 0 : (a < nt ? a : nt);
    }
    return nt;
}


// Misfit epilogue of the inverse transform (see k_c2r).
struct MisfitArgs {
    const void* d_obs;       // [outer][t][col], I/O type
    const double* var;       // noise variances
    int var_mode;            // 0: scalar, 1: per column (sensor), 2: per (t, col)
    double* partials;
};

enum { EPI_PLAIN = 0, EPI_MISFIT = 1 };

}  // namespace p2o
