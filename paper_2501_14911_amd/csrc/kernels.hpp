// Internal launchers between the plan (abi.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include "common.hpp"

namespace p2o {

struct GemvArgs {
    int Nd;
    int pitch;            // complex entries per stored row (>= Nm, multiple of 32): row stride
    int ncols;            // columns that can be nonzero (Nm rounded up to 8): the column extent
    int nfreq;
    int nrhs;
    int nblk;             // scale blocks per row
    int nslab;            // row slabs (adjoint: partial outputs; forward: row tiling)
    int rows_per_wg;      // rows per slab
    long long part_stride;  // complex elements between partial outputs
};

struct GemmArgs {
    int Nd;
    int pitch;            // complex entries per stored spectrum row (row stride)
    int ncols;            // columns that can be nonzero (Nm rounded up to 8): K extent / adjoint outputs
    int nfreq;
    int nrhs;
    int nblk;
    long long part_stride;  // complex elements between forward partial outputs
    int a_f16;              // spectrum words are FP16 (re, im) pairs (BF16 otherwise); LDS-ring tiles only
    const float* rhs_scale; // FP16 spectra: per-right-hand-side power-of-two scales of the complex FP32 operand
    // FP16 operands of the data-space columns (FP16 spectra, LDS-ring tiles):
    // the adjoint writes its products as FP16 (re, im) pairs multiplied by
    // out_scale[b] (when non-null); the forward reads such pairs as its
    // right-hand sides (b_f16, already scaled by rhs_scale[b]; tiles 13, 14)
    const float* out_scale;
    int b_f16;
    // filled in by the launcher
    int ldb;                // complex values per right-hand-side row of the quad B operand
    int kchunk;             // complex columns per forward K chunk
    int n_kc, n_mt, n_bg;   // K chunks, row (or column) tiles, right-hand-side groups
    int items, Q;           // work items and items per XCD
};

struct LoadArgs {
    void* fhat;
    float* scales;        // [nfreq][nblk]
    unsigned* flag;       // non-finite flag
    long long col0;
    int ncols;
    int Nd;
    int Nt;
    long long t_stride;   // elements between time steps of the source chunk (Nd * ncols)
    long long pitch;
    int nblk;
    int rows_per_wg;
};

// fft.hip
int fft_tile_shift(int M, bool f64);
// Tile shift of the compiled-length kernels' wide tiles for this plan and
// precision (used for transforms of at least kWideSeries series), or -1.
int fixed_wide_shift(bool f64, const FftPlan& pl);
// Wavefronts per workgroup of the compiled-length kernels for tile shift sh
// (4 where no compiled case has that shift): one per-tile maximum slot each.
int fixed_tile_waves(bool f64, const FftPlan& pl, int sh);
// Truncate-and-repad of FP16 operands (see launch_project_half), or false;
// err == nullptr only reports whether a kernel exists.
bool launch_fixed_project_h(const FftPlan& pl, const SeriesIO& io, void* in_out, const void* tw, int sh,
                            const float* sx, const float* sy, hipStream_t st, hipError_t* err);
// In-place truncate-and-repad of FP16 (re, im) pairs: input multiplied by
// sx[outer], output by sy[outer]; the compiled-length kernels only (false,
// and nothing launched, without one; err == nullptr: availability only).
bool launch_project_half(const FftPlan& pl, const SeriesIO& io, void* in_out, const void* tw, const float* sx,
                         const float* sy, hipStream_t st, hipError_t* err);
constexpr int kWideSeries = 2048;
int c2r_grid_x(const FftPlan& pl, bool f64, int S);
hipError_t launch_twiddle(void* tw64, void* tw32, int L, hipStream_t st);
hipError_t launch_r2c(bool f64, bool in_f64, const FftPlan& pl, const SeriesIO& io, const void* in, void* out,
                      const void* tw, hipStream_t st);
hipError_t launch_c2r(bool f64, const FftPlan& pl, const SeriesIO& io, const void* in, void* out, const void* tw,
                      const void* d_obs, const double* var, int var_mode, double* partials, hipStream_t st);
hipError_t launch_project(bool f64, const FftPlan& pl, const SeriesIO& io, void* in_out, const void* tw,
                          hipStream_t st);
hipError_t launch_misfit_reduce(const double* partials, int nper, double* misfit, int nrhs, hipStream_t st);
hipError_t launch_load(int prec, bool in_f64, const FftPlan& pl, const LoadArgs& la, const void* in,
                       const void* tw64, hipStream_t st);
hipError_t launch_zero_pad(void* fhat, long long rows, int pitch, int Nm, int bytes, hipStream_t st);
int load_tile_shift(int M);
int fft_amax_slots(int S_pad);   // wavefront-maximum slots per outer index a transform of S_pad series needs

// fft_fixed.hip: kernels compiled for fixed transform lengths.  Each returns
// false when there is none for (M, tile shift, precision) or the plan turned
// them off (pl.fixed == 0); otherwise it launches and sets *err.
bool launch_fixed_r2c(bool f64, bool in_f64, const FftPlan& pl, const SeriesIO& io, const void* in, void* out,
                      const void* tw, int sh, hipStream_t st, hipError_t* err);
bool launch_fixed_c2r(bool f64, const FftPlan& pl, const SeriesIO& io, const void* in, void* out, const void* tw,
                      int sh, const void* d_obs, const double* var, int var_mode, double* partials, hipStream_t st,
                      hipError_t* err);
bool launch_fixed_project(bool f64, const FftPlan& pl, const SeriesIO& io, void* in_out, const void* tw, int sh,
                          hipStream_t st, hipError_t* err);

// gemv.hip
int gemv_cols_per_lane(int prec);
int gemv_fwd_chunks(int prec, int ncols);
hipError_t launch_gemv_fwd(int prec, const GemvArgs& ga, const void* fhat, const float* scales, const void* X,
                           void* Yp, hipStream_t st);
hipError_t launch_gemv_adj(int prec, const GemvArgs& ga, const void* fhat, const float* scales, const void* Y,
                           void* Xp, hipStream_t st);

// probe.hip
hipError_t launch_probe(int mode, const void* src, void* dst, size_t bytes, int blocks, hipStream_t st);

// gemm_mfma.hip
int gemm_fwd_kchunks(int ncols);
int gemm_data_pitch(int Nd);   // row length of data-side quad spectra read by the adjoint (Nd rounded up to 16)
int gemm_tile_count();
bool gemm_tile_has(int tile, bool fwd);   // variant exists for that direction (others take the built-in choice)
int gemm_tile_shape(int tile, int* row_groups, int* substeps, int* blocks, int* rhs_per_group);
int gemm_default_tile(int nrhs, bool fwd, int Nd);
bool gemm_tile_is_ring(int tile);           // an LDS-ring variant (the only ones for FP16 spectra)
bool gemm_f16_fits(int Nd, int pitch);      // shapes the FP16-spectrum ring kernels can address
hipError_t launch_fill_bf16(void* p, size_t bytes, uint32_t seed, hipStream_t st);   // timing operands
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t st);
// tile: a variant index, or -1 for the built-in choice
hipError_t launch_gemm_fwd(const GemmArgs& ga, int tile, const void* fhat, const float* scales, const void* Xq,
                           void* Yp, hipStream_t st);
hipError_t launch_gemm_adj(const GemmArgs& ga, int tile, const void* fhat, const float* scales, const void* Yq,
                           void* Xp, hipStream_t st);

// posterior.hip: data-space matrix, Cholesky factorisation and solves, and
// the elementwise steps of the online phase (dense matrices FP64,
// column-major; f64 selects FP64 series, FP32 otherwise)
hipError_t launch_unit_vectors(bool f64, void* E, long long N, long long j0, int ncols, double value, hipStream_t st);
hipError_t launch_K_columns(bool f64, const void* H, long long N, double* K, long long ldk, long long j0, int ncols,
                            const double* var, int var_mode, int Nd, hipStream_t st);
hipError_t launch_weight_data(bool f64, const void* d, void* D, long long N, int nrhs, const double* var, int var_mode,
                              int Nd, double gamma, hipStream_t st);
hipError_t launch_to_f64(bool f64, const void* Y, double* Z, long long N, int nrhs, long long ldz, hipStream_t st);
hipError_t launch_combine(bool f64, void* D, const double* Z, long long N, int nrhs, long long ldz, double a0, double a1,
                          hipStream_t st);
hipError_t launch_axpby(bool f64, const void* v, void* out, long long n, double a0, double a1, hipStream_t st);
hipError_t launch_qoi_scatter(bool f64, const void* q, void* Y, int Nt, int Nd, int r, int nrhs, hipStream_t st);
hipError_t launch_qoi_gather(bool f64, const void* Y, void* q, double* C, long long ldc, long long c0, double alpha,
                             bool accum, int Nt, int Nd, int r, int nrhs, hipStream_t st);
hipError_t launch_d2q_rows(bool f64, const void* y, const void* h, long long N, int nrows, double* Q, long long ldq,
                           long long r0, const double* var, int var_mode, int Nd, double gamma, hipStream_t st);
hipError_t launch_d2q_apply(const double* Q, long long nq, long long N, long long ldq, const double* d, double* q,
                            int nrhs, hipStream_t st);
// Power-of-two scales of the FP16 operands of a data-space column call, from
// its data-side spectra Y ([nfreq][nrhs][ld] complex FP32) and the spectrum's
// block multipliers: sx[b] for the adjoint's outputs, sy[b] for the
// re-padded right-hand sides; part holds nfreq nrhs floats of row bounds.
hipError_t launch_fp16_operand_scales(const void* Y, int ld, int nrhs, int nfreq, int Nd, const float* scales, int nblk,
                                      int Nt, float* part, float* sx, float* sy, hipStream_t st);
// G += B B^T (lower triangle; B: N rows of kc columns, row stride ldb), and
// K = prior_var (block-diagonal prefix sums of G) + Gamma_noise, mirrored.
hipError_t launch_gram_update(const double* B, long long ldb, long long N, int kc, double* G, long long ldg,
                              hipStream_t st);
hipError_t launch_gram_to_K(double* G, long long ldg, int Nt, int Nd, double prior_var, const double* var,
                            int var_mode, hipStream_t st);
hipError_t launch_cholesky(double* A, long long n, long long lda, int* info, hipStream_t st);
hipError_t launch_cholesky_solve(const double* L, long long n, long long lda, double* X, int nrhs, long long ldx,
                                 hipStream_t st);

}  // namespace p2o
