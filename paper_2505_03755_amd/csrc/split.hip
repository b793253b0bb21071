// Split-precision products on the int8 matrix cores of gfx950 (v_mfma_i32_16x16x64_i8).
//
// A FP64 row x[0..K) is written as
//     x[k] = 2^e * sum_{s < S} a_s[k] * 2^-(6 + 7 s)  +  r[k],   |r[k]| <= 2^(e - 7 - 7 (S - 1))
// with e the exponent of max|x| (max|x| < 2^e) and integer slices a_s in [-64, 64] stored as
// int8: a_0 = rint(x 2^-e 2^6); after each slice the residual (|.| <= 1/2) is scaled by 2^7 and
// rounded again.  Every step is exact in FP64 (power-of-two scalings, and a number minus its
// nearest integer).  Round-to-nearest keeps the truncation error zero-mean.
//
// The product of two split rows keeps the slice pairs with s + t <= S - 1 and groups them by
// d = s + t: sum_k a_s[k] b_t[k] is exact in int32 over 32768 k (|a b| <= 2^12, at most 8 pairs
// per d), after which the int32 sums are flushed into FP64 as F += 2^(-7 d) I_d.  The result is
// 2^(e_a + e_b - 12) F.
//
// Planes are [S][rows][kp] int8 with kp a multiple of 64 and zeros past K; exponents [rows] int32.
//
// Operand layout of v_mfma_i32_16x16x64_i8 (checked on gfx950): A[i][k] in lane i + 16 (k / 16),
// byte k % 16 (B likewise with its column j); D[i][j] in lane j + 16 (i / 4), element i % 4.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.h"

namespace dfk {

typedef int v4i __attribute__((ext_vector_type(4)));

namespace {

constexpr int kSplitBits0 = 6, kSplitBits = 7;

// Block index -> work item with runs of consecutive items on one XCD (the dispatcher deals
// consecutive workgroups to the 8 XCDs in turn).
__device__ __forceinline__ int64_t xcd_remap_i8(int64_t id, int64_t n) {
  const int64_t full = (n / 8) * 8;
  if (id >= full) return id;
  return (id % 8) * (full / 8) + id / 8;
}

__device__ __forceinline__ int row_exponent(double m) {
  int e = 0;
  if (m > 0.0) frexp(m, &e);   // m = f 2^e, f in [0.5, 1): m < 2^e
  return e;
}

// slices of x * 2^-e (|.| < 1), written to planes[s * plane + off]
template <int S>
__device__ __forceinline__ void write_slices(double x, int e, int8_t* planes, int64_t plane, int64_t off) {
  double r = ldexp(x, kSplitBits0 - e);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const double a = rint(r);
    planes[s * plane + off] = (int8_t)(int)a;
    r = (r - a) * (double)(1 << kSplitBits);
  }
}

// max |.| over one row, by one 256-thread workgroup
__device__ __forceinline__ double block_max(double v) {
  __shared__ double red[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int t = threadIdx.x;
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  v = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return v;
}

// Rows of a dense operand given as an OpMap; the contraction index k = kb * kc_n + kc runs over
// K = kb_n * kc_n.  Work is cut into chunks of kSplitChunk k per workgroup (grid x = chunk,
// y = row): one pass takes the chunk maxima into the row exponent with an integer atomic max
// (exponents order like the magnitudes), a second writes the slices, four k per thread as one
// 32-bit word per plane.
constexpr int kSplitChunk = 1024;
constexpr int kNoExponent = -1000;   // rows that are all zero keep this (their slices are 0)

__device__ __forceinline__ const double* opmap_row(const OpMap& o, int64_t r) {
  const int64_t rh = o.s_rh ? r / o.rl : 0, rlo = o.s_rh ? r % o.rl : r;
  return o.p + rh * o.s_rh + rlo * o.s_rlo;
}

// Walks k = (kb, kc) of one row in steps of `step` without dividing per element.
struct KWalk {
  int64_t kb, kc, db, dc, kc_n;
  __device__ __forceinline__ KWalk(const OpMap& o, int64_t k, int64_t step)
      : kb(k / o.kc_n), kc(k % o.kc_n), db(step / o.kc_n), dc(step % o.kc_n), kc_n(o.kc_n) {}
  __device__ __forceinline__ int64_t off(const OpMap& o) const { return kb * o.s_kb + kc * o.s_kc; }
  __device__ __forceinline__ void next() {
    kb += db;
    kc += dc;
    if (kc >= kc_n) {
      kc -= kc_n;
      ++kb;
    }
  }
};

__global__ void __launch_bounds__(256) fill_int_kernel(int* p, int64_t n, int v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) split_max_kernel(OpMap o, int64_t K, int64_t r0, int* ex) {
  const int64_t r = r0 + blockIdx.y, k0 = (int64_t)blockIdx.x * kSplitChunk;
  const double* row = opmap_row(o, r);
  double m = 0.0;
  KWalk w(o, k0 + threadIdx.x, 256);
  for (int64_t k = k0 + threadIdx.x; k < K && k < k0 + kSplitChunk; k += 256) {
    m = fmax(m, fabs(row[w.off(o)]));
    w.next();
  }
  m = block_max(m);
  if (threadIdx.x == 0 && m > 0.0) atomicMax(ex + r, row_exponent(m));
}

template <int S>
__global__ void __launch_bounds__(256) split_slice_kernel(OpMap o, int64_t K, int64_t kp, int64_t r0, int8_t* planes,
                                                          const int* ex) {
  const int64_t r = r0 + blockIdx.y, k = (int64_t)blockIdx.x * kSplitChunk + 4 * threadIdx.x;
  if (k >= kp) return;
  const double* row = opmap_row(o, r);
  const int e = ex[r];
  const int64_t plane = o.rows * kp;
  double x[4];
  KWalk w(o, k < K ? k : 0, 1);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    x[q] = k + q < K ? ldexp(row[w.off(o)], kSplitBits0 - e) : 0.0;
    w.next();
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    uint32_t w = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double a = rint(x[q]);
      w |= ((uint32_t)(int)a & 0xffu) << (8 * q);
      x[q] = (x[q] - a) * (double)(1 << kSplitBits);
    }
    *(uint32_t*)(planes + s * plane + r * kp + k) = w;
  }
}

// Row (P, m) of the unpacked b^P: element k = b^P_{mk}, packed at T(max) + min.
template <int S>
__global__ void __launch_bounds__(256) split_packed_kernel(const double* __restrict__ B, int64_t nao, int64_t npair,
                                                           int64_t kp, int8_t* planes, int* ex, int64_t rows) {
  const int64_t r = blockIdx.x;
  const int64_t P = r / nao, m = r % nao;
  const double* Bp = B + P * npair;
  const int t = threadIdx.x;
  auto elem = [&](int64_t k) {
    const int64_t hi = m > k ? m : k, lo = m > k ? k : m;
    return Bp[hi * (hi + 1) / 2 + lo];
  };
  double mx = 0.0;
  for (int64_t k = t; k < nao; k += 256) mx = fmax(mx, fabs(elem(k)));
  const int e = row_exponent(block_max(mx));
  if (t == 0) ex[r] = e;
  const int64_t plane = rows * kp;
  for (int64_t k = t; k < kp; k += 256) write_slices<S>(k < nao ? elem(k) : 0.0, e, planes, plane, r * kp + k);
}

// ---------------------------------------------------------------------------------------
// Slice product.  Workgroup tile 64 x 64 over 8 waves (2 x 4) of 32 x 16 (two MFMA tiles), k steps
// of 64 bytes through one LDS stage refilled from registers between two barriers; the global
// loads of the next step are in flight while the current one is multiplied.  About 200
// registers per lane: two waves per SIMD, accumulators in VGPRs.  With `tri`, only tiles
// I >= J of a square output are formed (the lower half of a symmetric product).
constexpr int kTM = 64, kKB = 64, kRow = 80;   // LDS row pitch 80 bytes: conflict-free operand reads
constexpr int kFlushSteps = 512;               // 32768 k per int32 accumulation

template <int S>
struct I8Tile {
  static constexpr int LDS = 2 * S * kTM * kRow;   // A then B, slices outer
};

template <int S, bool GEN>
__global__ void __launch_bounds__(512) slice_gemm_kernel(const int8_t* __restrict__ Ap, const int* __restrict__ ea,
                                                         int64_t M, const int8_t* __restrict__ Bp,
                                                         const int* __restrict__ eb, int64_t N, int64_t kp,
                                                         OutMap O, int64_t tilesM, int64_t tilesN, int tri,
                                                         int64_t ntri, double* part) {
  __shared__ __attribute__((aligned(16))) int8_t lds[I8Tile<S>::LDS];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave & 1, wn = wave >> 1;      // rows 32 wm.., columns 16 wn..
  const int nsplit = gridDim.y, split = blockIdx.y;
  int64_t I, J;
  if (tri) {
    const int64_t pr = xcd_remap_i8(blockIdx.x, ntri);
    I = (int64_t)((sqrt(8.0 * (double)pr + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > pr) --I;
    while ((I + 1) * (I + 2) / 2 <= pr) ++I;
    J = pr - I * (I + 1) / 2;
  } else {
    // column tiles of one row block side by side (on one XCD): the row block is read once
    const int64_t tile = xcd_remap_i8(blockIdx.x, tilesM * tilesN);
    I = tile / tilesN;
    J = tile % tilesN;
  }
  const int64_t m0 = I * kTM, n0 = J * kTM;
  const int64_t nks = kp / kKB;
  const int64_t ks0 = nks * split / nsplit, ks1 = nks * (split + 1) / nsplit;

  // global -> register staging: threads 0..255 load A, 256..511 load B: 16 bytes of row
  // (t % 256) / 4, chunk t % 4, of every slice
  const int side = t >> 8, lr = (t & 255) >> 2, lc = (t & 3) * 16;
  const int64_t rows = side ? N : M, r0 = side ? n0 : m0;
  const int64_t rr = r0 + lr < rows ? r0 + lr : rows - 1;
  const int64_t plane = rows * kp;
  const int8_t* g = (side ? Bp : Ap) + rr * kp + lc;
  int8_t* lw = lds + (side * S * kTM + lr) * kRow + lc;
  // two register stages: the loads of step k + 2 go out while step k + 1 is still in flight
  v4i st[2][S];
  auto gload = [&](int b, int64_t ks) {
#pragma unroll
    for (int s = 0; s < S; ++s) st[b][s] = *(const v4i*)(g + s * plane + ks * kKB);
  };
  auto lstore = [&](int b) {
#pragma unroll
    for (int s = 0; s < S; ++s) *(v4i*)(lw + s * kTM * kRow) = st[b][s];
  };

  v4i acc[S][2];
  double F[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) F[i][r] = 0.0;

  // operand fragment reads: row / column (lane % 16) of a 16-row tile, bytes 16 (lane / 16)
  const int fr = lane & 15, fk = (lane >> 4) * 16;
  const int8_t* la = lds + (wm * 32 + fr) * kRow + fk;
  const int8_t* lb = lds + (S * kTM + wn * 16 + fr) * kRow + fk;
  // one k step: registers of stage b to LDS, refill stage b with step ks + 2, multiply
  auto step = [&](int b, int64_t ks) {
    __syncthreads();   // the previous step's reads of LDS are done
    lstore(b);
    __syncthreads();
    if (ks + 2 < ks1) gload(b, ks + 2);
    v4i fb[S];
#pragma unroll
    for (int s = 0; s < S; ++s) fb[s] = *(const v4i*)(lb + s * kTM * kRow);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      v4i fa[S];
#pragma unroll
      for (int s = 0; s < S; ++s) fa[s] = *(const v4i*)(la + (s * kTM + i * 16) * kRow);
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int u = 0; u + s < S; ++u)
          acc[s + u][i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[s], fb[u], acc[s + u][i], 0, 0, 0);
    }
  };
  if (ks1 > ks0) gload(0, ks0);
  if (ks1 > ks0 + 1) gload(1, ks0 + 1);
  for (int64_t kc = ks0; kc < ks1; kc += kFlushSteps) {   // chunks start at even offsets from ks0
    const int64_t kend = kc + kFlushSteps < ks1 ? kc + kFlushSteps : ks1;
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
      for (int i = 0; i < 2; ++i) acc[d][i] = v4i{0, 0, 0, 0};
    for (int64_t ks = kc; ks < kend; ks += 2) {
      step(0, ks);
      if (ks + 1 < kend) step(1, ks + 1);
    }
    // int32 sums of this chunk into FP64
#pragma unroll
    for (int d = 0; d < S; ++d)
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) F[i][r] += ldexp((double)acc[d][i][r], -kSplitBits * d);
  }

  // epilogue: value = 2^(ea + eb - 12) F
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t m = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + r;
      const int64_t n = n0 + wn * 16 + (lane & 15);
      if (m >= M || n >= N) continue;
      const double val = ldexp(F[i][r], ea[m] + eb[n] - 2 * kSplitBits0);
      if (part) {
        part[((int64_t)split * M + m) * N + n] = val;
      } else {
        double* dst;
        if (n < O.nsplit) {
          const int64_t nh = O.s_nh ? n / O.nl : 0, mh = O.s_mh ? m / O.ml : 0;
          dst = O.p + (mh * O.s_mh + (m - mh * O.ml) * O.s_ml) + (nh * O.s_nh + (n - nh * O.nl) * O.s_nl);
        } else {
          dst = O.p2 + m * O.s2_m + (n - O.nsplit);
        }
        if (GEN) *dst = O.accumulate ? *dst + O.alpha * val : O.alpha * val;
        else *dst = val;
      }
    }
}

}  // namespace

int64_t kpad64(int64_t n) { return (n + 63) / 64 * 64; }

template <int S>
static hipError_t split_rows_s(const OpMap& o, int64_t K, int8_t* planes, int* ex, hipStream_t s) {
  const int64_t kp = kpad64(K);
  fill_int_kernel<<<(unsigned)((o.rows + 255) / 256), 256, 0, s>>>(ex, o.rows, kNoExponent);
  for (int64_t r0 = 0; r0 < o.rows; r0 += 65535) {   // grid y carries the row
    const unsigned nr = (unsigned)(o.rows - r0 < 65535 ? o.rows - r0 : 65535);
    split_max_kernel<<<dim3((unsigned)((K + kSplitChunk - 1) / kSplitChunk), nr), 256, 0, s>>>(o, K, r0, ex);
  }
  for (int64_t r0 = 0; r0 < o.rows; r0 += 65535) {
    const unsigned nr = (unsigned)(o.rows - r0 < 65535 ? o.rows - r0 : 65535);
    split_slice_kernel<S><<<dim3((unsigned)((kp + kSplitChunk - 1) / kSplitChunk), nr), 256, 0, s>>>(o, K, kp, r0,
                                                                                                      planes, ex);
  }
  return hipGetLastError();
}

hipError_t launch_split_rows(const OpMap& o, int64_t K, int nslice, int8_t* planes, int* ex, hipStream_t s) {
  if (o.rows <= 0) return hipSuccess;
  if (o.rows > 0x7fffffffLL || K <= 0 || (kpad64(K) + kSplitChunk - 1) / kSplitChunk > 0x7fffffffLL)
    return hipErrorInvalidValue;
  switch (nslice) {
    case 4: return split_rows_s<4>(o, K, planes, ex, s);
    case 5: return split_rows_s<5>(o, K, planes, ex, s);
    case 6: return split_rows_s<6>(o, K, planes, ex, s);
    case 7: return split_rows_s<7>(o, K, planes, ex, s);
    case 8: return split_rows_s<8>(o, K, planes, ex, s);
    default: return hipErrorInvalidValue;
  }
}

template <int S>
static hipError_t split_packed_s(const double* B, int64_t naux, int64_t nao, int8_t* planes, int* ex,
                                 hipStream_t s) {
  const int64_t rows = naux * nao;
  split_packed_kernel<S><<<(unsigned)rows, 256, 0, s>>>(B, nao, nao * (nao + 1) / 2, kpad64(nao), planes, ex, rows);
  return hipGetLastError();
}

hipError_t launch_split_packed(const double* B, int64_t naux, int64_t nao, int nslice, int8_t* planes, int* ex,
                               hipStream_t s) {
  const int64_t rows = naux * nao;
  if (rows <= 0) return hipSuccess;
  if (rows > 0x7fffffffLL) return hipErrorInvalidValue;
  switch (nslice) {
    case 4: return split_packed_s<4>(B, naux, nao, planes, ex, s);
    case 5: return split_packed_s<5>(B, naux, nao, planes, ex, s);
    case 6: return split_packed_s<6>(B, naux, nao, planes, ex, s);
    case 7: return split_packed_s<7>(B, naux, nao, planes, ex, s);
    case 8: return split_packed_s<8>(B, naux, nao, planes, ex, s);
    default: return hipErrorInvalidValue;
  }
}

template <int S>
static void slice_gemm_s(const int8_t* A, const int* ea, int64_t M, const int8_t* B, const int* eb, int64_t N,
                         int64_t kp, const OutMap& O, bool tri, int nsplit, double* part, hipStream_t s) {
  const int64_t tm = (M + kTM - 1) / kTM, tn = (N + kTM - 1) / kTM;
  const int64_t ntri = tm * (tm + 1) / 2;
  const dim3 grid((unsigned)(tri ? ntri : tm * tn), (unsigned)nsplit, 1);
  const bool gen = !part && (O.alpha != 1.0 || O.accumulate);
  if (gen) slice_gemm_kernel<S, true><<<grid, 512, 0, s>>>(A, ea, M, B, eb, N, kp, O, tm, tn, tri, ntri, part);
  else slice_gemm_kernel<S, false><<<grid, 512, 0, s>>>(A, ea, M, B, eb, N, kp, O, tm, tn, tri, ntri, part);
}

hipError_t launch_slice_gemm(const int8_t* A, const int* ea, int64_t M, const int8_t* B, const int* eb, int64_t N,
                             int64_t kp, int nslice, const OutMap& O, bool tri, int nsplit, double* part,
                             hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (kp % 64 != 0 || kp <= 0 || nsplit < 1 || nsplit > 65535 || (tri && M != N) || (nsplit > 1 && !part))
    return hipErrorInvalidValue;
  const int64_t tm = (M + kTM - 1) / kTM, tn = (N + kTM - 1) / kTM;
  if ((tri ? tm * (tm + 1) / 2 : tm * tn) > 0x7fffffffLL) return hipErrorInvalidValue;
  switch (nslice) {
    case 4: slice_gemm_s<4>(A, ea, M, B, eb, N, kp, O, tri, nsplit, part, s); break;
    case 5: slice_gemm_s<5>(A, ea, M, B, eb, N, kp, O, tri, nsplit, part, s); break;
    case 6: slice_gemm_s<6>(A, ea, M, B, eb, N, kp, O, tri, nsplit, part, s); break;
    case 7: slice_gemm_s<7>(A, ea, M, B, eb, N, kp, O, tri, nsplit, part, s); break;
    case 8: slice_gemm_s<8>(A, ea, M, B, eb, N, kp, O, tri, nsplit, part, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int slice_gemm_tile() { return kTM; }

}  // namespace dfk
