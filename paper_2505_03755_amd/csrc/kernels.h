// Internal launcher interface between the C-ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dfk {

// Element (r, k) of a matrix operand in batch z.  The row index r in [0, rows) splits as
// r = rh * rl + rlo; the contraction index k splits as (kb, kc), kb in [0, kb_n),
// kc in [0, kc_n).  Address = p + z*s_z + kb*s_kb + (rh*s_rh + rlo*s_rlo + kc*s_kc).
// The bracketed part must stay below 2^32 elements (offsets_fit on the host).
struct OpMap {
  const double* p;
  int64_t rows, rl, s_rh, s_rlo;
  int64_t kb_n, kc_n, s_kb, s_kc;
  int64_t s_z;
  const double* ks;   // optional per-contraction-index scale: element *= ks[z*s_ksz + kc]
  int64_t s_ksz;
};

// Output element (m, n) of batch z.  Columns n < nsplit go to
//   p + z*s_z + (m/ml)*s_mh + (m%ml)*s_ml + (n/nl)*s_nh + (n%nl)*s_nl,
// columns n >= nsplit to  p2 + z*s2_z + m*s2_m + (n - nsplit).
// The stored value is alpha * result, added to what is there when `accumulate` is set.
struct OutMap {
  double* p;
  int64_t M, N;
  int64_t ml, s_mh, s_ml;
  int64_t nl, s_nh, s_nl;
  int64_t s_z;
  int64_t nsplit;
  double* p2;
  int64_t s2_m, s2_z;
  double alpha;
  int accumulate;
};

__host__ __device__ inline OpMap op_map(const double* p, int64_t rows, int64_t ld_row, int64_t kc_n, int64_t ld_k) {
  // element (r, k) at p + r*ld_row + k*ld_k
  return OpMap{p, rows, rows > 0 ? rows : 1, 0, ld_row, 1, kc_n, 0, ld_k, 0, nullptr, 0};
}

__host__ __device__ inline OutMap out_plain(double* p, int64_t M, int64_t N, int64_t ld) {
  return OutMap{p, M, N, M > 0 ? M : 1, 0, ld, N > 0 ? N : 1, 0, 1, 0, N, nullptr, 0, 0, 1.0, 0};
}

// True when every within-slab element offset of `o` fits 32 bits.
bool offsets_fit(const OpMap& o);

// n rounded up to a multiple of the 16-deep contraction slab.
inline int64_t kpad16(int64_t n) { return (n + 15) / 16 * 16; }

// Half transform: for each P, T[m][c] = sum_k b^P_{mk} C[k][c], c in [0, ncol), written
// through `out` with z = P (out.M = nao, out.N = ncol; alpha and accumulate honoured).  C has
// kpad16(nao) rows (row stride ldc), rows nao.. zero.
hipError_t launch_half_transform(const double* B, int64_t naux, int64_t nao, const double* C, int64_t ldc,
                                 int64_t ncol, const OutMap& out, hipStream_t s);
// The same with the J-vector of Eq. (J_1) formed in its epilogue: v[P] = sum_{m<nao, c<nv}
// T[m][c] C[m][c] w[c] over the first nv columns (w NULL: all ones; added to v when `accumulate`).
// Per-tile partial sums go to part [naux][half_tiles(nao, ncol)] first.  out.alpha must be 1 and
// out.accumulate 0.
int64_t half_tiles(int64_t nao, int64_t ncol);
hipError_t launch_half_transform_jvec(const double* B, int64_t naux, int64_t nao, const double* C, int64_t ldc,
                                      int64_t ncol, const OutMap& out, const double* w, int64_t nv, double* part,
                                      double* v, int accumulate, hipStream_t s);

// C(m, n) = sum_k A(m, k) B(n, k) for a batch of nz problems (grid z).
hipError_t launch_gemm(const OpMap& A, const OpMap& Bm, const OutMap& C, int64_t nz, hipStream_t s);

// The same product for one problem with the contraction split over nsplit workgroup sets:
// partial sums go to part [nsplit][M][N] and a fixed-order reduction writes C.  gemm_splits()
// is the split count the workspace is planned with (part needs nsplit*M*N doubles if > 1).
int gemm_splits(int64_t M, int64_t N, int64_t nslab);
// The most splits gemm_splits(M, N, s) gives for any s <= nslab (a bound for sizing partials).
int gemm_splits_bound(int64_t M, int64_t N, int64_t nslab);
int64_t gemm_slabs(const OpMap& A);
hipError_t launch_gemm_split(const OpMap& A, const OpMap& Bm, const OutMap& C, int nsplit, double* part,
                             hipStream_t s);

// C = alpha * sum_s part[s] (+ C), fixed order over s; part is [nsplit][O.M][O.N].
hipError_t launch_split_reduce(const double* part, int nsplit, const OutMap& O, hipStream_t s);

// C(m, n) = sum_{P < naux} sum_k b^P_{mk} Y(n, (P, k)), Y given as an OpMap whose kb is P and
// kc the AO index k (kc_n = nao); for every P the entries k in [nao, kpad16(nao)) must exist
// and be zero.  The P range is split over workgroups, each piece of the tiling with its own
// split count, and the partials (in `part`, half_reduce_part_bound(nao, N, naux) doubles at most)
// are added up in a fixed order.  C must have no row or column blocking (s_mh = s_nh = 0).
int64_t half_reduce_part_bound(int64_t nao, int64_t N, int64_t naux);
hipError_t launch_half_reduce(const double* B, int64_t naux, int64_t nao, const OpMap& Y, const OutMap& C,
                              double* part, hipStream_t s);

// g[pair(i,j)] = G[i][j] + G[j][i] (i > j), G[i][i] (i == j): <b^P, G> = sum_pair b^P[pair] g[pair]
hipError_t launch_pair_weights(const double* G, int64_t nao, double* g, hipStream_t s);
// Dw [ndm][npair] = the packed densities C_z C_z^T of C [ndm][nao][nocc], off-diagonal pairs
// weighted 2 (so that v[z][P] = sum_pair b^P[pair] Dw[z][pair]); D [ndm][nao][nao] is scratch
// for the full products.  ndm <= 65535.
hipError_t launch_dens_pairs(const double* C, int64_t nao, int64_t nocc, int64_t ndm, double* D, double* Dw,
                             hipStream_t s);
// u[P] = sum_pair B[P][pair] g[pair]
// (partial sums over jvec_packed_chunks() chunks of the pairs go to part [chunks][naux] first)
int jvec_packed_chunks();
hipError_t launch_jvec_packed(const double* B, int64_t naux, int64_t nao, const double* g, double* part, double* u,
                              hipStream_t s);
// out[z] = in[z] + in[z]^T for nz square n x n matrices (out may equal in)
hipError_t launch_symmetrize(const double* in, int64_t n, int64_t nz, double* out, hipStream_t s);

// Lower-tile SYRK with a split over kb: Kpart[split][z][i][j] = sum_{kb in split, kc} A(i,(kb,kc)) Bw(j,(kb,kc))
// for tile(i) >= tile(j) (Bw = A with an optional per-kc weight).  Kpart is dense [nsplit][nz][n][n];
// syrk_splits() gives the number of splits the workspace is planned for.
int syrk_splits(int64_t n, int64_t kb_n, int64_t nz);
// The most splits syrk_splits(n, k, nz) gives for any k <= kb_n.
int syrk_splits_bound(int64_t n, int64_t kb_n, int64_t nz);
// SYRK tile edge for an n x n result (64 up to n = 640, else 128); a group uses the edge of its
// largest member.
int syrk_tile_for(int64_t n);
hipError_t launch_syrk_partial(const OpMap& A, const OpMap& Bw, int64_t n, int64_t nz, int nsplit,
                               double* Kpart, hipStream_t s);
// K[z][i][j] = sum_s Kpart[s][z][max(i,j)][min(i,j)]; both triangles written (added to K
// when `accumulate`).
hipError_t launch_syrk_reduce(const double* Kpart, int nsplit, int64_t n, int64_t nz, double* K,
                              hipStream_t s, int accumulate = 0);

// v[z][P] = sum_{m<nao, c<nocc} C[z][m][c] w[z][c] X[P][m][z*nocc + c]   (X row stride ldx; v row
// stride ldv, naux when 0; added to v when `accumulate`)
hipError_t launch_jvec(const double* X, int64_t naux, int64_t nao, int64_t ldx, const double* C,
                       const double* w, int64_t nocc, int64_t nz, double* v, hipStream_t s, int accumulate = 0,
                       int64_t ldv = 0);

// J[z][i][j] = sum_P v[z][P] b^P_{ij}, both triangles written (added to J when `accumulate`; v row
// stride ldv, naux when 0).
hipError_t launch_coulomb(const double* B, int64_t naux, int64_t nao, const double* v,
                          int64_t nz, double* J, hipStream_t s, int accumulate = 0, int64_t ldv = 0);
// y[r][c] = x[r][c] (or += with `accumulate`) for x [rows][cols] contiguous, y of row stride ldy
hipError_t launch_copy_rows(const double* x, int64_t rows, int64_t cols, double* y, int64_t ldy, int accumulate,
                            hipStream_t s);

// y[i] += x[i], i < n
hipError_t launch_add(const double* x, int64_t n, double* y, hipStream_t s);
// Xw[i] = X[i] * w[i % ncol], i < n (columns of a row-major [n / ncol][ncol] matrix scaled)
hipError_t launch_scale_cols(const double* X, int64_t n, int64_t ncol, const double* w, double* Xw, hipStream_t s);

// p[0..n) = 0
hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t s);
// J[z][i][j] = J[z][j][i] = Jp[z][pair(i, j)] for nz packed symmetric matrices
hipError_t launch_unpack_sym(const double* Jp, int64_t nz, int64_t nao, double* J, hipStream_t s);
// Diagonal-block edge of the blocked metric Cholesky.
constexpr int kCholNB = 128;
// Factor the kb x kb block at A (row stride lda; kb <= kCholNB) in place: lower triangle = its
// Cholesky factor, strictly upper part zeroed; Linv [kCholNB][kCholNB] = the factor's inverse
// (lower).  info: 0 written when `first`, then k0 + j + 1 for a pivot j that is not positive
// unless an earlier one is recorded.  One workgroup.
hipError_t launch_chol_block(double* A, int64_t lda, int kb, double* Linv, int* info, int64_t k0, bool first,
                             hipStream_t s);
// A[i][j] = 0 for j > i (n x n, row major)
hipError_t launch_zero_upper(double* A, int64_t n, hipStream_t s);
// Ap[z][pair(i, j)] = A[z][i][j] for i >= j: the lower triangles of nz n x n matrices, packed
hipError_t launch_pack_lower(const double* A, int64_t nz, int64_t n, double* Ap, hipStream_t s);
// p[z*s_z + i] = 0 for z < nz, i < n
hipError_t launch_fill_zero_strided(double* p, int64_t nz, int64_t s_z, int64_t n, hipStream_t s);

// ---- grouped launches over several problems (at most 8 per launch, largest first) ----
// problems per grouped launch (their descriptors travel in the kernel arguments)
constexpr int kMaxGroup = 8;
// Half transform of problem p: as launch_half_transform with (B, naux, nao, C, ldc, ncol, out).
struct GroupHalf {
  const double* B;
  int64_t naux, nao;
  const double* C;   // kpad16(nao) rows, zero past nao
  int64_t ldc, ncol;
  OutMap out;
};
// tile_n: column tile of the launch on one row of waves, 176, 96 or 48 (0 = 176); or 128: the
// 2-D tiling (128 x 128 tiles on 2 x 2 waves of 4 x 4 MFMA blocks, and per problem, where the
// padded area says it pays, the rows past its last whole 128-row band on 64 x 176 tiles in a
// second grouped launch).
hipError_t launch_half_group(const GroupHalf* probs, int n, int tile_n, hipStream_t s);
// The tile_n of launch_half_group with the least estimated time (padded area over matrix-core
// busy fraction) over problems of nao[i] rows and ncol[i] columns: 128 or 176.
int half_group_tile_for(const int64_t* nao, const int64_t* ncol, int n);
// Lower-tile SYRK partials of problem p: as launch_syrk_partial with (A, A, n, nz, nsplit, Kpart).
struct GroupSyrk {
  OpMap A;
  int64_t n, nz;
  int nsplit;
  double* Kpart;
};
// tile: 64 or 128 (0 = syrk_group_tile()).
hipError_t launch_syrk_group(const GroupSyrk* probs, int n, int tile, hipStream_t s);
int syrk_group_tile(const GroupSyrk* probs, int n);

// ---- split precision (split.hip) ----
// n rounded up to a multiple of 64 (contraction length of the planes) and of 32 (their rows).
int64_t kpad64(int64_t n);
int64_t rpad32(int64_t n);
// Bytes of the planes of an operand: nslice * rpad32(rows) * kpad64(K), in 1 KB blocks of 32 rows
// x 32 k; block (s, g, b) at ((s * G + g) * KB + b) KB (G = rpad32(rows) / 32, KB = kpad64(K) / 32),
// slot l = rr + 32 c (16 bytes) of it holding k = 32 b + 16 c + [0, 16) of row 32 g + rr.
int64_t split_plane_bytes(int64_t rows, int64_t K, int nslice);
// Splits each row r < o.rows of the operand (k over kb_n * kc_n = K) into nslice int8 planes
// (zeros past K and past o.rows) and its exponent ex[r].  nslice in [4, 8].
hipError_t launch_split_rows(const OpMap& o, int64_t K, int nslice, int8_t* planes, int* ex, hipStream_t s);
// The same for nz operands in one launch set (grid z): operand z at o.p + z o.s_z, its planes at
// planes + z plane_stride, its exponents at ex + z ex_stride (ex_stride >= o.rows).  nz <= 65535.
hipError_t launch_split_rows_batched(const OpMap& o, int64_t K, int nslice, int8_t* planes, int* ex, int64_t nz,
                                     int64_t plane_stride, int64_t ex_stride, hipStream_t s);
// The same for the rows (P, m) of the unpacked b^P (rows naux*nao, K = nao).
hipError_t launch_split_packed(const double* B, int64_t naux, int64_t nao, int nslice, int8_t* planes, int* ex,
                               hipStream_t s);
// The same for the rows mu of the DF tensor over k = (P, nu), k = P nao + nu (rows nao,
// K = naux * nao): the exponent of row mu is the largest over P.
hipError_t launch_split_packed_t(const double* B, int64_t naux, int64_t nao, int nslice, int8_t* planes, int* ex,
                                 hipStream_t s);
// C(m, n) = sum_k A(m, k) B(n, k) from the split planes of A (M rows) and B (N rows) with
// kp = kpad64(K), written through O (alpha / accumulate honoured) or, with nsplit > 1, as partial
// sums part[split][M][N] over k ranges.  Every split must be at most slice_gemm_max_steps() steps
// of 32 k long (the int32 sums are exact up to there).  With tri (M == N) tiles wholly above the
// diagonal are skipped; the tiles on it are written whole.
hipError_t launch_slice_gemm(const int8_t* A, const int* ea, int64_t M, const int8_t* B, const int* eb, int64_t N,
                             int64_t kp, int nslice, const OutMap& O, bool tri, int nsplit, double* part,
                             hipStream_t s);
// A batch of nz slice products of equal shape: product z reads A + z a, ea + z ea, B + z b,
// eb + z eb (bytes of planes, entries of exponents) and writes O at z O.s_z (z O.s2_z for the
// columns past O.nsplit) or partials part[split][z][M][N].
struct SliceBatch {
  int64_t a, ea, b, eb;
};
hipError_t launch_slice_gemm_batched(const int8_t* A, const int* ea, int64_t M, const int8_t* B, const int* eb,
                                     int64_t N, int64_t kp, int nslice, const OutMap& O, bool tri, int nsplit,
                                     double* part, int64_t nz, const SliceBatch& zs, hipStream_t s);
// Workgroup tiles of a slice product that do work, 32-deep steps of a contraction of kp, and
// the longest split in steps.
int64_t slice_gemm_tiles(int64_t M, int64_t N, bool tri);
int64_t slice_gemm_steps(int64_t kp);
int64_t slice_gemm_max_steps();

}  // namespace dfk
