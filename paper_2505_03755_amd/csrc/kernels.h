// Internal launcher interface between the C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dfk {

// Element (r, k) of a matrix operand.  The row index r in [0, rows) splits as
// r = rh * rl + rlo; the contraction index k splits as (kb, kc), kb in [0, kb_n),
// kc in [0, kc_n).  Address = p + rh*s_rh + rlo*s_rlo + kb*s_kb + kc*s_kc (+ z*s_z).
struct OpMap {
  const double* p;
  int64_t rows, rl, s_rh, s_rlo;
  int64_t kb_n, kc_n, s_kb, s_kc;
  int64_t s_z;
  const double* ks;   // optional per-contraction-index scale: element *= ks[z*s_ksz + kc]
  int64_t s_ksz;
};

// Output element (m, n): p + z*s_z + (m/ml)*s_mh + (m%ml)*s_ml + (n/nl)*s_nh + (n%nl)*s_nl.
struct OutMap {
  double* p;
  int64_t M, N;
  int64_t ml, s_mh, s_ml;
  int64_t nl, s_nh, s_nl;
  int64_t s_z;
};

__host__ __device__ inline OpMap op_rowmajor(const double* p, int64_t rows, int64_t k, int64_t ld_row, int64_t ld_k) {
  // element (r, k) at p + r*ld_row + k*ld_k
  return OpMap{p, rows, rows > 0 ? rows : 1, 0, ld_row, 1, k, 0, ld_k, 0, nullptr, 0};
}

__host__ __device__ inline OutMap out_plain(double* p, int64_t M, int64_t N, int64_t ld) {
  return OutMap{p, M, N, M > 0 ? M : 1, 0, ld, N > 0 ? N : 1, 0, 1, 0};
}

// X[P][m][c] = sum_k b^P_{mk} C[k][c] for c in [0, ncol); X row stride ldx, slab stride
// nao*ldx.  P in [p0, p0 + np_).
hipError_t launch_half_transform(const double* B, int64_t naux, int64_t nao, const double* C,
                                 int64_t ldc, int64_t ncol, double* X, int64_t ldx,
                                 hipStream_t s);

// C(m, n) = sum_k A(m, k) B(n, k) for a batch of nz problems (grid z).
hipError_t launch_gemm(const OpMap& A, const OpMap& Bm, const OutMap& C, int64_t nz, hipStream_t s);

// Lower-tile SYRK with a split over kb: Kpart[split][z][i][j] = sum_{kb in split, kc} A(i,(kb,kc)) A(j,(kb,kc))
// for tile(i) >= tile(j).  Returns the number of splits used through *nsplit (planning:
// syrk_splits()).  Kpart is dense [nsplit][nz][n][n].
int syrk_splits(int64_t n, int64_t kb_n, int64_t nz);
int syrk_tile();
// Bw is A with an optional contraction-index scale (signed occupation weights).
hipError_t launch_syrk_partial(const OpMap& A, const OpMap& Bw, int64_t n, int64_t nz, int nsplit,
                               double* Kpart, hipStream_t s);
// K[z][i][j] = sum_s Kpart[s][z][max-tile element]; both triangles written.
hipError_t launch_syrk_reduce(const double* Kpart, int nsplit, int64_t n, int64_t nz, double* K,
                              hipStream_t s);

// v[z][P] = sum_{m<nao, c<nocc} C[z][m][c] w[z][c] X[P][m][z*nocc + c]   (X row stride ldx)
hipError_t launch_jvec(const double* X, int64_t naux, int64_t nao, int64_t ldx, const double* C,
                       const double* w, int64_t nocc, int64_t nz, double* v, hipStream_t s);

// J[z][i][j] = sum_P v[z][P] b^P_{ij}, both triangles written.
hipError_t launch_coulomb(const double* B, int64_t naux, int64_t nao, const double* v,
                          int64_t nz, double* J, hipStream_t s);

// Y[r][c] = 0 for a strided 2-D block (used for zero-sized contractions).
hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t s);

}  // namespace dfk
