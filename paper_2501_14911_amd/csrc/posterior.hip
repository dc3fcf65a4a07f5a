// Kernels of the offline and online phases built on the p2o map (section 4,
// Phases 2-4): assembly of the data-space matrix K = Gamma_noise + F G*
// from batched operator columns, its Cholesky factorisation K = L L^T, the
// triangular solves with L, and the small elementwise steps of the MAP point
// and posterior-covariance actions.
//
// Dense matrices are FP64 and column-major with a leading dimension: entry
// (i, j) at A[j * lda + i].  The data-space index is j = t * Nd + s (the
// time-major order of the data series).
//
// Cholesky (right-looking, panels of kNB2 = 256 columns made of blocks of
// kNB = 64):
//   for each 64-column block k of a panel: factor its diagonal block in
//   registers (one wavefront, lane r holding row r); solve the rows below
//   it against L_kk^T (one row per lane, L_kk in LDS); subtract its P P^T
//   from the panel's remaining columns.  After the panel: subtract the
//   panel's rank-256 product from the lower tiles of the trailing matrix.
//   Both updates run on v_mfma_f64_16x16x4f64 (128 x 128 tiles, the panel
//   columns staged in LDS 16 at a time, the tile accumulated in registers
//   and written once).
// The factor is also written transposed into the strict upper triangle
// (entry (i, j), i < j, receives L(j, i)), so that both triangular solves
// read whole contiguous column runs: the forward solve columns of L, the
// backward solve columns of L^T.
#include "common.hpp"
#include "kernels.hpp"

namespace p2o {

namespace {

constexpr int kNB = 64;                 // Cholesky / solve block size
constexpr int kNB2 = 256;               // Cholesky panel width (trailing updates of rank kNB2)
constexpr int kLP = kNB + 2;            // padded LDS row (doubles)

__device__ __forceinline__ double noise_var_at(const double* var, int mode, long long i, int Nd) {
    return mode == 0 ? var[0] : mode == 1 ? var[i % Nd] : var[i];
}

// ---------------------------------------------------------------- K assembly
// E[b][i] = value at i = j0 + b, zero elsewhere (b < ncols, i < N).
template <typename T>
__global__ void k_unit_vectors(T* __restrict__ E, long long N, long long j0, int ncols, T value) {
    const long long n = N * ncols;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long b = e / N, i = e - b * N;
        E[e] = (i == j0 + b) ? value : T(0);
    }
}

// K[:, j0 + b] = H[b] + Gamma_noise e_{j0+b}: the operator columns (FP32 or
// FP64) widened to FP64, the noise variance added on the diagonal.
template <typename T>
__global__ void k_K_columns(const T* __restrict__ H, long long N, double* __restrict__ K, long long ldk, long long j0,
                            int ncols, const double* __restrict__ var, int var_mode, int Nd) {
    const long long n = N * ncols;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long b = e / N, i = e - b * N;
        double v = (double)H[e];
        if (i == j0 + b) v += noise_var_at(var, var_mode, i, Nd);
        K[(j0 + b) * ldk + i] = v;
    }
}

// ---------------------------------------------------------------- elementwise steps of the online phase
// D = gamma d / var (nrhs data series of N values).
template <typename T>
__global__ void k_weight_data(const T* __restrict__ d, T* __restrict__ D, long long N, int nrhs,
                              const double* __restrict__ var, int var_mode, int Nd, double gamma) {
    const long long n = N * nrhs;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long i = e % N;
        D[e] = (T)(gamma * (double)d[e] / noise_var_at(var, var_mode, i, Nd));
    }
}

// Z[b][i] = Y[b][i] widened to FP64 (Z rows ldz apart).
template <typename T>
__global__ void k_to_f64(const T* __restrict__ Y, double* __restrict__ Z, long long N, int nrhs, long long ldz) {
    const long long n = N * nrhs;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long b = e / N, i = e - b * N;
        Z[b * ldz + i] = (double)Y[e];
    }
}

// D[b][i] = a0 * D[b][i] + a1 * Z[b][i]   (Z rows ldz apart).
// (a0 = 0 does not read D, so stale contents never reach the result.)
template <typename T>
__global__ void k_combine(T* __restrict__ D, const double* __restrict__ Z, long long N, int nrhs, long long ldz,
                          double a0, double a1) {
    const long long n = N * nrhs;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long b = e / N, i = e - b * N;
        const double z = a1 * Z[b * ldz + i];
        D[e] = (T)(a0 == 0.0 ? z : a0 * (double)D[e] + z);
    }
}

// out = a0 * out + a1 * v (a0 = 0 does not read out).
template <typename T>
__global__ void k_axpby(const T* __restrict__ v, T* __restrict__ out, long long n, double a0, double a1) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const double y = a1 * (double)v[e];
        out[e] = (T)(a0 == 0.0 ? y : a0 * (double)out[e] + y);
    }
}

// ---------------------------------------------------------------- multi-rate (QoI) series
// A plan observed every r-th step (QoI series, section 2 remark on distinct
// temporal discretisations; section 5: QoIs at 1 Hz, parameters at 10 Hz)
// exchanges series of Nt / r steps, step i standing for fine step r (i+1) - 1.
// Y[b][t][s] = q[b][t / r][s] at those steps, 0 elsewhere.
template <typename T>
__global__ void k_qoi_scatter(const T* __restrict__ q, T* __restrict__ Y, int Nt, int Nd, int r, int nrhs) {
    const long long n = (long long)nrhs * Nt * Nd;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long b = e / ((long long)Nt * Nd);
        const int rem = (int)(e - b * Nt * Nd), t = rem / Nd, s = rem - t * Nd;
        Y[e] = (t % r == r - 1) ? q[(b * (Nt / r) + t / r) * Nd + s] : T(0);
    }
}

// q[b][i][s] = Y[b][r (i + 1) - 1][s]; with f64 output (C given), column
// c0 + b of C (leading dimension ldc) receives alpha q[b] (added when accum).
template <typename T>
__global__ void k_qoi_gather(const T* __restrict__ Y, T* __restrict__ q, double* __restrict__ C, long long ldc,
                             long long c0, double alpha, int accum, int Nt, int Nd, int r, int nrhs) {
    const int Ntq = Nt / r;
    const long long n = (long long)nrhs * Ntq * Nd;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long b = e / ((long long)Ntq * Nd);
        const int rem = (int)(e - b * Ntq * Nd), i = rem / Nd, s = rem - i * Nd;
        const T v = Y[(b * Nt + (long long)r * (i + 1) - 1) * Nd + s];
        if (C) {
            double* c = C + (c0 + b) * ldc + rem;
            *c = accum ? *c + alpha * (double)v : alpha * (double)v;
        } else {
            q[e] = v;
        }
    }
}

// Rows r0 + b of the data-to-QoI map: Q[(r0 + b) ldq + i] =
// gamma (y[b][i] - h[b][i]) / var_i.
template <typename T>
__global__ void k_d2q_rows(const T* __restrict__ y, const T* __restrict__ h, long long N, int nrows,
                           double* __restrict__ Q, long long ldq, long long r0, const double* __restrict__ var,
                           int var_mode, int Nd, double gamma) {
    const long long n = N * nrows;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const long long b = e / N, i = e - b * N;
        Q[(r0 + b) * ldq + i] = gamma * ((double)y[e] - (double)h[e]) / noise_var_at(var, var_mode, i, Nd);
    }
}

// q[b][r] = sum_j Q[r ldq + j] d[b][j]: one wavefront per (row, right-hand
// side), lanes striding over j (coalesced), fixed-order reduction.
__global__ __launch_bounds__(256) void k_d2q_apply(const double* __restrict__ Q, long long nq, long long N,
                                                   long long ldq, const double* __restrict__ d, double* __restrict__ q,
                                                   int nrhs) {
    const long long w = blockIdx.x * 4LL + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= nq * nrhs) return;
    const long long r = w % nq, b = w / nq;
    const double* row = Q + r * ldq;
    const double* x = d + b * N;
    double acc = 0.0;
    for (long long j = lane; j < N; j += 64) acc += row[j] * x[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) q[b * nq + r] = acc;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane), hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// ---------------------------------------------------------------- Cholesky
// Factor the nb x nb diagonal block at (k, k) in place (nb <= kNB), one
// wavefront: lane r keeps row r of the block in registers; for each column
// j the pivot is broadcast from lane j, the column is scaled, and its outer
// product leaves the trailing part (row c of the column broadcast from lane
// c).  Entries right of the diagonal in the registers are never stored.  A
// pivot that is not positive (or not a number) records k + j + 1 in *info
// if nothing was recorded before (*info is reset by the call with k = 0).
// L is also written transposed into the upper triangle of the block.
__global__ __launch_bounds__(64) void k_potrf_diag(double* __restrict__ A, long long lda, int k, int nb,
                                                   int* __restrict__ info) {
    const int r = threadIdx.x;
    const int prev = (info && k > 0) ? *info : 0;
    double a[kNB];
#pragma unroll
    for (int c = 0; c < kNB; ++c) a[c] = (c <= r && r < nb) ? A[(long long)(k + c) * lda + k + r] : 0.0;
    int bad = 0;                                       // first non-positive pivot of the block (1-based)
#pragma unroll
    for (int j = 0; j < kNB; ++j) {
        if (j < nb) {
            const double d = readlane_f64(a[j], j);
            if (!(d > 0.0) && bad == 0) bad = j + 1;
            const double piv = sqrt(d), inv = 1.0 / piv;
            a[j] = r == j ? piv : (r > j ? a[j] * inv : 0.0);
#pragma unroll
            for (int c = j + 1; c < kNB; ++c) a[c] -= a[j] * readlane_f64(a[j], c);
        }
    }
    if (r < nb) {
#pragma unroll
        for (int c = 0; c < kNB; ++c) {
            if (c <= r) A[(long long)(k + c) * lda + k + r] = a[c];
            if (c < r) A[(long long)(k + r) * lda + k + c] = a[c];    // L^T in the upper triangle
        }
    }
    if (r == 0 && info) {
        if (k == 0) *info = bad;
        else if (prev == 0 && bad) *info = k + bad;
    }
}

// Rows r in [k + kNB, n) of the panel: x L_kk^T = a for each row (forward
// substitution along the row), one row per lane, L_kk staged in LDS.
__global__ __launch_bounds__(256) void k_trsm_panel(double* __restrict__ A, long long lda, int n, int k) {
    __shared__ double l[kNB][kLP];                     // l[col][row] = L_kk(row, col)
    for (int e = threadIdx.x; e < kNB * kNB; e += 256) {
        const int c = e / kNB, r = e - c * kNB;
        l[c][r] = r >= c ? A[(long long)(k + c) * lda + k + r] : 0.0;
    }
    __syncthreads();
    const long long r = (long long)k + kNB + blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    double x[kNB];
#pragma unroll
    for (int c = 0; c < kNB; ++c) x[c] = A[(long long)(k + c) * lda + r];
#pragma unroll
    for (int j = 0; j < kNB; ++j) {
        double s = x[j];
#pragma unroll
        for (int c = 0; c < j; ++c) s -= x[c] * l[c][j];
        x[j] = s / l[j][j];
    }
#pragma unroll
    for (int c = 0; c < kNB; ++c) A[(long long)(k + c) * lda + r] = x[c];
#pragma unroll
    for (int c = 0; c < kNB; ++c) A[r * lda + k + c] = x[c];           // L^T: row k + c, column r
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Update A[t0 + i, t0 + j] -= sum_c P[i, c] P[j, c] over the 128 x 128
// tiles of rows [t0, n) and columns [t0, c_end) on or below the diagonal
// (tile row >= tile column), P = A[t0:n, pk0:pk0 + kd].  Workgroup = one
// tile, 4 wavefronts of 64 x 64 (4 x 4 blocks of 16 x 16 on the matrix
// cores), accumulated in registers and written once.  The panel columns
// pass through LDS kKC at a time; the next columns are loaded into
// registers while the matrix cores work on the current ones.  The products
// are taken as the transposed block P_j P_i^T so that lane l of a block
// holds rows l % 16 of four columns: stores cover 128 contiguous bytes per
// 16 lanes.  Tiles are numbered column by column: column tile tj has T - tj
// tiles (T row tiles).
constexpr int kST = 128;                // update tile
constexpr int kKC = 16;                 // panel columns per LDS stage
constexpr int kSP = kST + 2;            // padded LDS row (doubles)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_syrk_update(double* __restrict__ A, long long lda, int n, int t0, int c_end,
                                                     int pk0, int kd) {
    __shared__ double pi[kKC][kSP], pj[kKC][kSP];     // [panel column][tile row]
    const int m = n - t0, mc = c_end - t0;
    const int T = (m + kST - 1) / kST;
    // tile (ti, tj): tj is the largest column with S(tj) = tj (2T - tj + 1) / 2 <= q
    const long long q = blockIdx.x;
    const double b2 = 2.0 * T + 1.0;
    int tj = (int)((b2 - sqrt(b2 * b2 - 8.0 * (double)q)) * 0.5);
    auto S = [&](long long c) { return c * (2LL * T - c + 1) / 2; };
    while (tj > 0 && S(tj) > q) --tj;
    while (S(tj + 1) <= q) ++tj;
    const int ti = tj + (int)(q - S(tj));
    const int ri = ti * kST, rj = tj * kST;            // first rows (relative to t0)
    if (rj >= mc) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;   // sub-tile: rows wr (of i), columns wc (of j)
    const int li = lane & 15, lk = lane >> 4;
    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    // staging: thread t moves entries e = t + 256 u (column e / kST, row e % kST) of both panels
    constexpr int NU = kKC * kST / 256;
    double si[NU], sj[NU];
    auto load = [&](int k0) {
        const int kw = min(kKC, kd - k0);
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int e = threadIdx.x + 256 * u, c = e / kST, r = e % kST;
            const double* col = A + (long long)(pk0 + k0 + c) * lda + t0;
            si[u] = c < kw && ri + r < m ? col[ri + r] : 0.0;
            sj[u] = c < kw && rj + r < m ? col[rj + r] : 0.0;
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int e = threadIdx.x + 256 * u, c = e / kST, r = e % kST;
            pi[c][r] = si[u];
            pj[c][r] = sj[u];
        }
    };
    load(0);
    stage();
    __syncthreads();
    for (int k0 = 0; k0 < kd; k0 += kKC) {
        const bool more = k0 + kKC < kd;
        if (more) load(k0 + kKC);                      // in flight during the products
#pragma unroll 2
        for (int c0 = 0; c0 < kKC; c0 += 4) {
            double vi[4], vj[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) vi[a] = pi[c0 + lk][wr + 16 * a + li];
#pragma unroll
            for (int b = 0; b < 4; ++b) vj[b] = pj[c0 + lk][wc + 16 * b + li];
            // block (a, b) of P_j P_i^T: rows = tile columns wc + 16 b + ., columns = tile rows wr + 16 a + .
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(vj[b], vi[a], acc[a][b], 0, 0, 0);
        }
        if (more) {
            __syncthreads();                           // every wavefront is done with these columns
            stage();
            __syncthreads();
        }
    }
    // lane l holds D[4 v + l / 16][l % 16] of each block in item v (measured
    // on gfx950 with an in-bounds probe): D row = j offset, D column = i offset
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = ri + wr + 16 * a + li;              // row of A (relative to t0)
                const int gj = rj + wc + 16 * b + 4 * v + lk;      // column of A
                if (gi < m && gj < mc && gi >= gj) {
                    double* p = A + (long long)(t0 + gj) * lda + t0 + gi;
                    *p -= acc[a][b][v];
                }
            }
}

static long long trapezoid_tiles(long long m, long long mc) {
    const long long T = (m + kST - 1) / kST, C = std::min(T, (mc + kST - 1) / kST);
    return C * (2 * T - C + 1) / 2;
}

// ---------------------------------------------------------------- K from the blocks' Gram matrix
// With the blocks F_k themselves at hand (not only their spectrum), the
// (i, j) block of F F^* is sum_{k <= min(i, j)} F_{i-k} F_{j-k}^T (F is
// block lower-triangular Toeplitz), i.e. for i >= j the sum over l <= j of
// G(i - j + l, l), G(p, q) = F_p F_q^T: prefix sums along the block
// diagonals of the Gram matrix G = A A^T of the stacked blocks
// A = [F_0; ...; F_{Nt-1}] (row t Nd + s = sensor s of F_t).  G is summed
// over column chunks of A as they are generated.

// G += B B^T on the lower 128 x 128 tiles (tile row >= tile column) of the
// N x N matrix G, B a chunk of A: N rows of kc columns, row r at B + r ldb.
// Tiling, register prefetch of the next 16 columns and matrix-core products
// as in k_syrk_update; the staging reads 16 consecutive columns (one 128-byte
// line) of each row.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void k_gram_update(const double* __restrict__ B, long long ldb, int N, int kc, double* __restrict__ G, long long ldg) {
    __shared__ double pi[kKC][kSP], pj[kKC][kSP];     // [chunk column][tile row]
    const int T = (N + kST - 1) / kST;
    const long long q = blockIdx.x;
    const double b2 = 2.0 * T + 1.0;
    int tj = (int)((b2 - sqrt(b2 * b2 - 8.0 * (double)q)) * 0.5);
    auto S = [&](long long c) { return c * (2LL * T - c + 1) / 2; };
    while (tj > 0 && S(tj) > q) --tj;
    while (S(tj + 1) <= q) ++tj;
    const int ti = tj + (int)(q - S(tj));
    const int ri = ti * kST, rj = tj * kST;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    const int li = lane & 15, lk = lane >> 4;
    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    // staging: thread t moves row e / kKC, column e % kKC, e = t + 256 u
    constexpr int NU = kKC * kST / 256;
    double si[NU], sj[NU];
    auto load = [&](int k0) {
        const int kw = min(kKC, kc - k0);
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int e = threadIdx.x + 256 * u, r = e / kKC, c = e % kKC;
            si[u] = c < kw && ri + r < N ? B[(long long)(ri + r) * ldb + k0 + c] : 0.0;
            sj[u] = c < kw && rj + r < N ? B[(long long)(rj + r) * ldb + k0 + c] : 0.0;
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int e = threadIdx.x + 256 * u, r = e / kKC, c = e % kKC;
            pi[c][r] = si[u];
            pj[c][r] = sj[u];
        }
    };
    load(0);
    stage();
    __syncthreads();
    for (int k0 = 0; k0 < kc; k0 += kKC) {
        const bool more = k0 + kKC < kc;
        if (more) load(k0 + kKC);
#pragma unroll 2
        for (int c0 = 0; c0 < kKC; c0 += 4) {
            double vi[4], vj[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) vi[a] = pi[c0 + lk][wr + 16 * a + li];
#pragma unroll
            for (int b = 0; b < 4; ++b) vj[b] = pj[c0 + lk][wc + 16 * b + li];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(vj[b], vi[a], acc[a][b], 0, 0, 0);
        }
        if (more) {
            __syncthreads();
            stage();
            __syncthreads();
        }
    }
    // lane l holds D[4 v + l / 16][l % 16]: D row = column offset of G, D column = row offset
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = ri + wr + 16 * a + li;
                const int gj = rj + wc + 16 * b + 4 * v + lk;
                if (gi < N && gj < N && gi >= gj) G[(long long)gj * ldg + gi] += acc[a][b][v];
            }
}

// Prefix sums along the block diagonals of the lower triangle of G, in
// place: thread (d, p, q) walks block (d + j, j), j = 0 .. Nt - 1 - d, entry
// (p, q), keeping the running sum in a register (q <= p on the diagonal
// blocks, whose upper parts are not computed).
__global__ void k_gram_prefix(double* __restrict__ G, long long ldg, int Nt, int Nd) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long per = (long long)Nd * Nd;
    if (t >= (long long)Nt * per) return;
    const int d = (int)(t / per), e = (int)(t % per), q = e / Nd, p = e % Nd;
    if (d == 0 && p < q) return;
    double* g = G + (long long)q * ldg + (long long)d * Nd + p;    // block (d, 0), entry (p, q)
    const long long step = (long long)Nd * ldg + Nd;                 // to block (d + j + 1, j + 1)
    double sum = 0.0;
    for (int j = 0; j < Nt - d; ++j) {
        sum += *g;
        *g = sum;
        g += step;
    }
}

// K from the prefix-summed G: K = prior_var G + Gamma_noise on and below the
// diagonal, mirrored into the upper triangle (64 x 64 tiles through LDS;
// tile (ti, tj), ti >= tj, writes its transpose to tile (tj, ti)).
__global__ __launch_bounds__(256) void k_gram_finish(double* __restrict__ G, long long ldg, int N, double prior_var,
                                                     const double* __restrict__ var, int var_mode, int Nd) {
    __shared__ double t[64][65];
    const long long qd = blockIdx.x;
    int ti = (int)((sqrt(8.0 * (double)qd + 1.0) - 1.0) * 0.5);
    while ((long long)(ti + 1) * (ti + 2) / 2 <= qd) ++ti;
    while ((long long)ti * (ti + 1) / 2 > qd) --ti;
    const int tj = (int)(qd - (long long)ti * (ti + 1) / 2);
    const int r0 = ti * 64, c0 = tj * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int c = e / 64, r = e % 64, i = r0 + r, j = c0 + c;
        if (i < N && j < N && i >= j) {
            double v = prior_var * G[(long long)j * ldg + i];
            if (i == j) v += noise_var_at(var, var_mode, i, Nd);
            G[(long long)j * ldg + i] = v;
            t[c][r] = v;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e / 64, c = e % 64, i = r0 + r, j = c0 + c;      // write K(j, i) = K(i, j), i > j
        if (i < N && j < N && i > j) G[(long long)i * ldg + j] = t[c][r];
    }
}

// ---------------------------------------------------------------- triangular solves with L
// Diagonal block k (nb rows) of the solves: X[b][k:k+nb] = L_kk^{-1} X[b][k:k+nb]
// (forward) or L_kk^{-T} X[b][k:k+nb] (backward).  One workgroup per
// right-hand side: all 256 lanes stage L_kk in LDS (16 independent loads
// each; rows past nb get a unit diagonal), then the first wavefront keeps
// lane i's row of L_kk (forward) or of L_kk^T (backward) in registers and
// substitutes along the 64 rows, broadcasting each solved entry with
// v_readlane.
template <bool BWD>
__global__ __launch_bounds__(256) void k_trsv_diag(const double* __restrict__ L, long long lda, int k, int nb,
                                                   double* __restrict__ X, long long ldx) {
    __shared__ double l[kNB][kLP];                     // l[col][row] = L_kk(row, col)
#pragma unroll
    for (int u = 0; u < kNB * kNB / 256; ++u) {
        const int e = threadIdx.x + 256 * u, c = e / kNB, r = e % kNB;
        l[c][r] = (r < nb && c < nb && r >= c) ? L[(long long)(k + c) * lda + k + r] : (r == c ? 1.0 : 0.0);
    }
    __syncthreads();
    if (threadIdx.x >= 64) return;
    const int i = threadIdx.x;
    double row[kNB];                                   // strictly off-diagonal coefficients of lane i's row
#pragma unroll
    for (int c = 0; c < kNB; ++c) row[c] = BWD ? (c > i ? l[i][c] : 0.0) : (c < i ? l[c][i] : 0.0);
    const double inv = 1.0 / l[i][i];
    double* x = X + blockIdx.x * ldx + k;
    double xi = i < nb ? x[i] : 0.0;
#pragma unroll
    for (int s = 0; s < kNB; ++s) {
        const int j = BWD ? kNB - 1 - s : s;
        if (i == j) xi *= inv;
        xi -= row[j] * readlane_f64(xi, j);
    }
    if (i < nb) x[i] = xi;
}

// Rows [row0, row0 + nrows) of the solves' updates with the nb columns of
// block k: X[b][r] -= sum_c A[r, k + c] X[b][k + c].  Forward solve: rows
// below the block, A = L.  Backward solve: rows above the block, where the
// upper triangle holds L^T.  Either way column k + c is one contiguous run;
// one row per lane, one wavefront per 64 rows.
__global__ __launch_bounds__(64) void k_trsv_update(const double* __restrict__ A, long long lda, long long row0,
                                                    long long nrows, int k, int nb, double* __restrict__ X,
                                                    long long ldx, int nrhs) {
    __shared__ double xs[8][kNB];
    const long long r = blockIdx.x * 64 + threadIdx.x;
    const bool live = r < nrows;
    double a[kNB];
#pragma unroll
    for (int c = 0; c < kNB; ++c) a[c] = live && c < nb ? A[(long long)(k + c) * lda + row0 + r] : 0.0;
    for (int b0 = 0; b0 < nrhs; b0 += 8) {
        const int m = min(8, nrhs - b0);
        __syncthreads();
        for (int e = threadIdx.x; e < 8 * kNB; e += 64) {
            const int b = e / kNB, c = e % kNB;
            xs[b][c] = b < m && c < nb ? X[(long long)(b0 + b) * ldx + k + c] : 0.0;
        }
        __syncthreads();
        if (live) {
            for (int b = 0; b < m; ++b) {
                double acc = 0.0;
#pragma unroll
                for (int c = 0; c < kNB; ++c) acc += a[c] * xs[b][c];
                X[(long long)(b0 + b) * ldx + row0 + r] -= acc;
            }
        }
    }
}

// The same update for many right-hand sides as a product on the FP64 matrix
// cores: workgroup = 64 rows x 64 right-hand sides, 4 wavefronts of 32 x 32
// (2 x 2 blocks of 16 x 16), the block's 64 columns of A and the 64 x 64
// right-hand-side values staged in LDS.  Taken as the transposed product
// (right-hand side x row) so that 16 lanes update 16 consecutive rows of one
// right-hand side (128 contiguous bytes).
__global__ __launch_bounds__(256) void k_trsv_update_mfma(const double* __restrict__ A, long long lda, long long row0,
                                                         long long nrows, int k, int nb, double* __restrict__ X,
                                                         long long ldx, int nrhs) {
    __shared__ double sa[kNB][kLP], sx[kNB][kLP];     // sa[c][r] = A(row0 + r0 + r, k + c), sx[c][b] = X[b0 + b][k + c]
    const long long r0 = (long long)blockIdx.x * 64;
    const int b0 = blockIdx.y * 64;
    for (int e = threadIdx.x; e < 64 * kNB; e += 256) {
        const int c = e / 64, r = e % 64;
        sa[c][r] = c < nb && r0 + r < nrows ? A[(long long)(k + c) * lda + row0 + r0 + r] : 0.0;
        const int b = e / kNB, cc = e % kNB;
        sx[cc][b] = cc < nb && b0 + b < nrhs ? X[(long long)(b0 + b) * ldx + k + cc] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = (wave >> 1) * 32, wb = (wave & 1) * 32;   // rows wr.., right-hand sides wb..
    const int li = lane & 15, lk = lane >> 4;
    f64x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int c0 = 0; c0 < kNB; c0 += 4) {
        double vr[2], vb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) vr[a] = sa[c0 + lk][wr + 16 * a + li];
#pragma unroll
        for (int b = 0; b < 2; ++b) vb[b] = sx[c0 + lk][wb + 16 * b + li];
        // block (a, b): rows of D = right-hand sides wb + 16 b + ., columns = rows wr + 16 a + .
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(vb[b], vr[a], acc[a][b], 0, 0, 0);
    }
    // lane l holds D[4 v + l / 16][l % 16] of each block in item v
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const long long r = r0 + wr + 16 * a + li;
                const int rb = b0 + wb + 16 * b + 4 * v + lk;
                if (r < nrows && rb < nrhs) X[(long long)rb * ldx + row0 + r] -= acc[a][b][v];
            }
}

// Single-right-hand-side solves, one launch per 64-row block: kernel j
// applies block j - 1's solved entries (forward; block j + 1's, backward) to
// the rows of block j and solves block j (workgroup 0: one wavefront keeps
// row i of the block in lane i, as in k_trsv_diag), while the other
// workgroups apply the same entries to every row past block j (forward; above
// it, backward), one row per lane.  Each row thus receives block m's entries
// in the launch after block m was solved: from workgroup 0 if it belongs to
// the next block, from the others otherwise.  The backward solve reads the
// factor's transpose from the upper triangle, so every update reads
// contiguous column runs.
template <bool BWD>
__global__ __launch_bounds__(256) void k_trsv_fused(const double* __restrict__ L, long long lda, int n, int j,
                                                    double* __restrict__ X) {
    const int nblk = (n + kNB - 1) / kNB;
    const int k = j * kNB, nb = min(kNB, n - k);
    const int src = BWD ? j + 1 : j - 1;               // block whose solved entries are applied
    const bool apply = BWD ? src < nblk : src >= 0;
    const int ks = src * kNB, nbs = apply ? min(kNB, n - ks) : 0;
    __shared__ double xs[kNB];                         // the applied block's solved entries
    __shared__ double l[kNB][kLP];                     // workgroup 0: l[col][row] = L_kk(row, col)
    if (threadIdx.x < kNB) xs[threadIdx.x] = (int)threadIdx.x < nbs ? X[ks + threadIdx.x] : 0.0;
    if (blockIdx.x > 0) {
        // rows past block j (forward: [k + nb, n); backward: [0, k)); all 64 loads issued before the sum
        const long long r = BWD ? (long long)(blockIdx.x - 1) * 256 + threadIdx.x
                                : (long long)k + nb + (long long)(blockIdx.x - 1) * 256 + threadIdx.x;
        const bool live = apply && (BWD ? r < k : r < n);
        double a[kNB];
#pragma unroll
        for (int c = 0; c < kNB; ++c) a[c] = live && c < nbs ? L[(long long)(ks + c) * lda + r] : 0.0;
        __syncthreads();
        if (!live) return;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kNB; ++c) acc += a[c] * xs[c];
        X[r] -= acc;
        return;
    }
#pragma unroll
    for (int u = 0; u < kNB * kNB / 256; ++u) {
        const int e = threadIdx.x + 256 * u, c = e / kNB, r = e % kNB;
        l[c][r] = (r < nb && c < nb && r >= c) ? L[(long long)(k + c) * lda + k + r] : (r == c ? 1.0 : 0.0);
    }
    const int i = threadIdx.x;
    double xi = 0.0;
    if (i < kNB) {
        const bool live = apply && i < nb;
        double a[kNB];
#pragma unroll
        for (int c = 0; c < kNB; ++c) a[c] = live && c < nbs ? L[(long long)(ks + c) * lda + k + i] : 0.0;
        xi = i < nb ? X[k + i] : 0.0;
        __syncthreads();
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < kNB; ++c) acc += a[c] * xs[c];
        xi -= acc;
    } else {
        __syncthreads();
        return;
    }
    double row[kNB];
#pragma unroll
    for (int c = 0; c < kNB; ++c) row[c] = BWD ? (c > i ? l[i][c] : 0.0) : (c < i ? l[c][i] : 0.0);
    const double inv = 1.0 / l[i][i];
#pragma unroll
    for (int s = 0; s < kNB; ++s) {
        const int jj = BWD ? kNB - 1 - s : s;
        if (i == jj) xi *= inv;
        xi -= row[jj] * readlane_f64(xi, jj);
    }
    if (i < nb) X[k + i] = xi;
}

dim3 grid_for(long long n) { return dim3((unsigned)std::max<long long>(1, std::min<long long>(4096, (n + 255) / 256))); }

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_unit_vectors(bool f64, void* E, long long N, long long j0, int ncols, double value, hipStream_t st) {
    if (f64)
        hipLaunchKernelGGL(k_unit_vectors<double>, grid_for(N * ncols), dim3(256), 0, st, (double*)E, N, j0, ncols, value);
    else
        hipLaunchKernelGGL(k_unit_vectors<float>, grid_for(N * ncols), dim3(256), 0, st, (float*)E, N, j0, ncols,
                           (float)value);
    return hipGetLastError();
}

hipError_t launch_K_columns(bool f64, const void* H, long long N, double* K, long long ldk, long long j0, int ncols,
                            const double* var, int var_mode, int Nd, hipStream_t st) {
    if (f64)
        hipLaunchKernelGGL(k_K_columns<double>, grid_for(N * ncols), dim3(256), 0, st, (const double*)H, N, K, ldk, j0,
                           ncols, var, var_mode, Nd);
    else
        hipLaunchKernelGGL(k_K_columns<float>, grid_for(N * ncols), dim3(256), 0, st, (const float*)H, N, K, ldk, j0,
                           ncols, var, var_mode, Nd);
    return hipGetLastError();
}

hipError_t launch_weight_data(bool f64, const void* d, void* D, long long N, int nrhs, const double* var, int var_mode,
                              int Nd, double gamma, hipStream_t st) {
    if (f64)
        hipLaunchKernelGGL(k_weight_data<double>, grid_for(N * nrhs), dim3(256), 0, st, (const double*)d, (double*)D, N,
                           nrhs, var, var_mode, Nd, gamma);
    else
        hipLaunchKernelGGL(k_weight_data<float>, grid_for(N * nrhs), dim3(256), 0, st, (const float*)d, (float*)D, N,
                           nrhs, var, var_mode, Nd, gamma);
    return hipGetLastError();
}

hipError_t launch_to_f64(bool f64, const void* Y, double* Z, long long N, int nrhs, long long ldz, hipStream_t st) {
    if (f64)
        hipLaunchKernelGGL(k_to_f64<double>, grid_for(N * nrhs), dim3(256), 0, st, (const double*)Y, Z, N, nrhs, ldz);
    else
        hipLaunchKernelGGL(k_to_f64<float>, grid_for(N * nrhs), dim3(256), 0, st, (const float*)Y, Z, N, nrhs, ldz);
    return hipGetLastError();
}

hipError_t launch_combine(bool f64, void* D, const double* Z, long long N, int nrhs, long long ldz, double a0, double a1,
                          hipStream_t st) {
    if (f64)
        hipLaunchKernelGGL(k_combine<double>, grid_for(N * nrhs), dim3(256), 0, st, (double*)D, Z, N, nrhs, ldz, a0, a1);
    else
        hipLaunchKernelGGL(k_combine<float>, grid_for(N * nrhs), dim3(256), 0, st, (float*)D, Z, N, nrhs, ldz, a0, a1);
    return hipGetLastError();
}

hipError_t launch_axpby(bool f64, const void* v, void* out, long long n, double a0, double a1, hipStream_t st) {
    if (f64)
        hipLaunchKernelGGL(k_axpby<double>, grid_for(n), dim3(256), 0, st, (const double*)v, (double*)out, n, a0, a1);
    else
        hipLaunchKernelGGL(k_axpby<float>, grid_for(n), dim3(256), 0, st, (const float*)v, (float*)out, n, a0, a1);
    return hipGetLastError();
}

hipError_t launch_qoi_scatter(bool f64, const void* q, void* Y, int Nt, int Nd, int r, int nrhs, hipStream_t st) {
    const long long n = (long long)nrhs * Nt * Nd;
    if (f64)
        hipLaunchKernelGGL(k_qoi_scatter<double>, grid_for(n), dim3(256), 0, st, (const double*)q, (double*)Y, Nt, Nd, r,
                           nrhs);
    else
        hipLaunchKernelGGL(k_qoi_scatter<float>, grid_for(n), dim3(256), 0, st, (const float*)q, (float*)Y, Nt, Nd, r,
                           nrhs);
    return hipGetLastError();
}

hipError_t launch_qoi_gather(bool f64, const void* Y, void* q, double* C, long long ldc, long long c0, double alpha,
                             bool accum, int Nt, int Nd, int r, int nrhs, hipStream_t st) {
    const long long n = (long long)nrhs * (Nt / r) * Nd;
    if (f64)
        hipLaunchKernelGGL(k_qoi_gather<double>, grid_for(n), dim3(256), 0, st, (const double*)Y, (double*)q, C, ldc, c0,
                           alpha, accum ? 1 : 0, Nt, Nd, r, nrhs);
    else
        hipLaunchKernelGGL(k_qoi_gather<float>, grid_for(n), dim3(256), 0, st, (const float*)Y, (float*)q, C, ldc, c0,
                           alpha, accum ? 1 : 0, Nt, Nd, r, nrhs);
    return hipGetLastError();
}

hipError_t launch_d2q_rows(bool f64, const void* y, const void* h, long long N, int nrows, double* Q, long long ldq,
                           long long r0, const double* var, int var_mode, int Nd, double gamma, hipStream_t st) {
    if (f64)
        hipLaunchKernelGGL(k_d2q_rows<double>, grid_for(N * nrows), dim3(256), 0, st, (const double*)y, (const double*)h,
                           N, nrows, Q, ldq, r0, var, var_mode, Nd, gamma);
    else
        hipLaunchKernelGGL(k_d2q_rows<float>, grid_for(N * nrows), dim3(256), 0, st, (const float*)y, (const float*)h, N,
                           nrows, Q, ldq, r0, var, var_mode, Nd, gamma);
    return hipGetLastError();
}

hipError_t launch_d2q_apply(const double* Q, long long nq, long long N, long long ldq, const double* d, double* q,
                            int nrhs, hipStream_t st) {
    const long long waves = nq * nrhs;
    hipLaunchKernelGGL(k_d2q_apply, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, Q, nq, N, ldq, d, q, nrhs);
    return hipGetLastError();
}

hipError_t launch_gram_update(const double* B, long long ldb, long long N, int kc, double* G, long long ldg,
                              hipStream_t st) {
    if (N <= 0 || kc <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gram_update, dim3((unsigned)trapezoid_tiles(N, N)), dim3(256), 0, st, B, ldb, (int)N, kc, G,
                       ldg);
    return hipGetLastError();
}

hipError_t launch_gram_to_K(double* G, long long ldg, int Nt, int Nd, double prior_var, const double* var,
                            int var_mode, hipStream_t st) {
    const long long N = (long long)Nt * Nd, nthr = (long long)Nt * Nd * Nd;
    hipLaunchKernelGGL(k_gram_prefix, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, st, G, ldg, Nt, Nd);
    const long long T = (N + 63) / 64;
    hipLaunchKernelGGL(k_gram_finish, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, st, G, ldg, (int)N, prior_var,
                       var, var_mode, Nd);
    return hipGetLastError();
}

hipError_t launch_cholesky(double* A, long long n, long long lda, int* info, hipStream_t st) {
    for (long long K0 = 0; K0 < n; K0 += kNB2) {
        const long long pend = std::min<long long>(K0 + kNB2, n);      // end of the panel
        for (long long k = K0; k < pend; k += kNB) {
            const int nb = (int)std::min<long long>(kNB, n - k);
            hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(64), 0, st, A, lda, (int)k, nb, info);
            const long long below = n - k - nb;
            if (below <= 0) break;
            hipLaunchKernelGGL(k_trsm_panel, dim3((unsigned)((below + 255) / 256)), dim3(256), 0, st, A, lda, (int)n,
                               (int)k);
            if (k + kNB < pend)                            // the panel's remaining columns, all rows below
                hipLaunchKernelGGL(k_syrk_update, dim3((unsigned)trapezoid_tiles(below, pend - k - kNB)), dim3(256), 0,
                                   st, A, lda, (int)n, (int)(k + kNB), (int)pend, (int)k, kNB);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (pend < n)                                       // trailing matrix, rank kNB2
            hipLaunchKernelGGL(k_syrk_update, dim3((unsigned)trapezoid_tiles(n - pend, n - pend)), dim3(256), 0, st, A,
                               lda, (int)n, (int)pend, (int)n, (int)K0, (int)(pend - K0));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// Solve updates: one row per lane for few right-hand sides, the matrix-core
// product from 16 on.
constexpr int kTrsvMfmaRhs = 16;
static void trsv_update(const double* L, long long lda, long long row0, long long nrows, int k, int nb, double* X,
                        long long ldx, int nrhs, hipStream_t st) {
    if (nrhs >= kTrsvMfmaRhs)
        hipLaunchKernelGGL(k_trsv_update_mfma, dim3((unsigned)((nrows + 63) / 64), (unsigned)((nrhs + 63) / 64)),
                           dim3(256), 0, st, L, lda, row0, nrows, k, nb, X, ldx, nrhs);
    else
        hipLaunchKernelGGL(k_trsv_update, dim3((unsigned)((nrows + 63) / 64)), dim3(64), 0, st, L, lda, row0, nrows, k,
                           nb, X, ldx, nrhs);
}

hipError_t launch_cholesky_solve(const double* L, long long n, long long lda, double* X, int nrhs, long long ldx,
                                 hipStream_t st) {
    if (nrhs == 1) {
        const long long nblk = (n + kNB - 1) / kNB;
        for (long long j = 0; j < nblk; ++j) {
            const long long rest = n - std::min<long long>(n, (j + 1) * kNB);       // rows past block j
            hipLaunchKernelGGL(k_trsv_fused<false>, dim3((unsigned)(1 + (rest + 255) / 256)), dim3(256), 0, st, L,
                               lda, (int)n, (int)j, X);
        }
        for (long long j = nblk - 1; j >= 0; --j)
            hipLaunchKernelGGL(k_trsv_fused<true>, dim3((unsigned)(1 + (j * kNB + 255) / 256)), dim3(256), 0, st, L,
                               lda, (int)n, (int)j, X);
        return hipGetLastError();
    }
    for (long long k = 0; k < n; k += kNB) {
        const int nb = (int)std::min<long long>(kNB, n - k);
        hipLaunchKernelGGL(k_trsv_diag<false>, dim3(nrhs), dim3(256), 0, st, L, lda, (int)k, nb, X, ldx);
        const long long below = n - k - nb;
        if (below > 0) trsv_update(L, lda, k + nb, below, (int)k, nb, X, ldx, nrhs, st);
    }
    for (long long k = (n - 1) / kNB * kNB; k >= 0; k -= kNB) {
        const int nb = (int)std::min<long long>(kNB, n - k);
        hipLaunchKernelGGL(k_trsv_diag<true>, dim3(nrhs), dim3(256), 0, st, L, lda, (int)k, nb, X, ldx);
        if (k > 0) trsv_update(L, lda, 0, k, (int)k, nb, X, ldx, nrhs, st);
    }
    return hipGetLastError();
}

}  // namespace p2o
