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
// Planes are int8 in 1 KB blocks of 32 rows x 32 k (layout below); exponents [rows] int32.
//
// Operand layout of v_mfma_i32_32x32x32_i8 (checked on gfx950): A[i][k] in lane i + 32 (k / 16),
// byte k % 16 (B likewise with its column j); D[i][j] in lane j + 32 ((i / 4) % 2), element
// 4 (i / 8) + i % 4.  global_load_lds with 16 bytes puts lane l's data at the LDS address + 16 l.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.h"

namespace dfk {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

namespace {

constexpr int kSplitBits0 = 6, kSplitBits = 7;

// s_waitcnt immediate that waits until at most N vector-memory operations are outstanding
// (vmcnt in bits 3:0 and 15:14; expcnt and lgkmcnt at their maxima, i.e. not waited on)
template <int N>
struct kVmcnt {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  static constexpr int imm = (N & 15) | (((N >> 4) & 3) << 14) | (7 << 4) | (15 << 8);
};

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

// Plane layout.  The planes of an operand with `rows` rows and contraction length K hold
// rpad32(rows) rows (zeros past `rows`) and kp = kpad64(K) k (zeros past K), cut into 1 KB blocks
// of 32 rows x 32 k: block (s, g, b) of slice s, row group g, k block b starts at byte
// ((s * G + g) * KB + b) * 1024 (G = rpad32(rows) / 32, KB = kp / 32), and its 16-byte slot
// l = rr + 32 c holds the 16 k = 32 b + 16 c + [0, 16) of row 32 g + rr -- the operand fragment
// of matrix-core lane l.  A block is one contiguous 1 KB load and one conflict-free LDS read.
__device__ __forceinline__ int64_t block_offset(int s, int64_t g, int64_t b, int64_t G, int64_t KB) {
  return (((int64_t)s * G + g) * KB + b) * 1024;
}

// Rows of a dense operand given as an OpMap; the contraction index k = kb * kc_n + kc runs over
// K = kb_n * kc_n.  The exponent pass cuts each row into chunks of kSplitChunk k per workgroup
// (grid x = chunk, y = row) and takes the chunk maxima into the row exponent with an integer
// atomic max (exponents order like the magnitudes).
constexpr int kSplitChunk = 4096;
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

// Operand z of a batch at o.p + z o.s_z, exponents at ex + z exs.  Grid (k chunk, row, z), or with
// zfast (z, row, k chunk): then the workgroups dispatched together read the same rows and k of
// adjacent operands, which for the densities of one X_occ are adjacent column runs.
__global__ void __launch_bounds__(256) split_max_kernel(OpMap o, int64_t K, int64_t r0, int* ex, int64_t exs,
                                                        int zfast) {
  const int64_t z = zfast ? blockIdx.x : blockIdx.z, chunk = zfast ? blockIdx.z : blockIdx.x;
  o.p += z * o.s_z;
  ex += z * exs;
  const int64_t r = r0 + blockIdx.y, k0 = chunk * kSplitChunk;
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

// The same for operands whose rows are adjacent in memory (row stride 1, contraction index far
// apart): 32 rows x kSplitChunkR k per workgroup with the lanes along the rows, so that every
// load reads 32 consecutive rows.
constexpr int kSplitChunkR = 256;
__global__ void __launch_bounds__(256) split_max_rows_kernel(OpMap o, int64_t K, int64_t y0, int* ex, int64_t exs) {
  o.p += (int64_t)blockIdx.z * o.s_z;
  ex += (int64_t)blockIdx.z * exs;
  const int t = threadIdx.x, rr = t & 31, kk = t >> 5;
  const int64_t r = 32 * (int64_t)blockIdx.x + rr, k0 = (y0 + blockIdx.y) * kSplitChunkR;
  double m = 0.0;
  if (r < o.rows) {
    const double* row = opmap_row(o, r);
    KWalk w(o, k0 + kk, 8);
    for (int64_t k = k0 + kk; k < K && k < k0 + kSplitChunkR; k += 8) {
      m = fmax(m, fabs(row[w.off(o)]));
      w.next();
    }
  }
  // the 8 threads of a row: lanes rr and rr + 32 of each of the 4 waves
  m = fmax(m, __shfl_xor(m, 32));
  __shared__ double red[4][32];
  if ((t & 63) < 32) red[t >> 6][rr] = m;
  __syncthreads();
  if (t < 32) {
    m = fmax(fmax(red[0][t], red[1][t]), fmax(red[2][t], red[3][t]));
    if (r < o.rows && m > 0.0) atomicMax(ex + r, row_exponent(m));
  }
}

// 16 scaled values of one slot -> its 16 bytes in each of the S planes
template <int S>
__device__ __forceinline__ void write_slot(double (&x)[16], int8_t* planes, int64_t G, int64_t KB, int64_t g,
                                           int64_t b, int slot) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    v4i w = {0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const double a = rint(x[q]);
      w[q >> 2] |= (int)(((uint32_t)(int)a & 0xffu) << (8 * (q & 3)));
      x[q] = (x[q] - a) * (double)(1 << kSplitBits);
    }
    *(v4i*)(planes + block_offset(s, g, b, G, KB) + slot * 16) = w;
  }
}

// One workgroup per (row group g = blockIdx.x, 128 k); thread t fills slot (rr = t % 32,
// 16 k at 16 (t / 32)) of its block in every plane; rows past o.rows are zero.
template <int S>
__global__ void __launch_bounds__(256) split_slice_kernel(OpMap o, int64_t K, int64_t kp, int64_t y0, int8_t* planes,
                                                          const int* ex, int64_t ps, int64_t exs) {
  o.p += (int64_t)blockIdx.z * o.s_z;
  planes += (int64_t)blockIdx.z * ps;
  ex += (int64_t)blockIdx.z * exs;
  const int t = threadIdx.x, rr = t & 31;
  const int64_t g = blockIdx.x, kq = (y0 + blockIdx.y) * 8 + (t >> 5);   // 16-k chunk
  if (16 * kq >= kp) return;
  const int64_t r = 32 * g + rr, k = 16 * kq;
  double x[16];
  if (r < o.rows) {
    const double* row = opmap_row(o, r);
    const int e = ex[r];
    KWalk w(o, k < K ? k : 0, 1);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      x[q] = k + q < K ? ldexp(row[w.off(o)], kSplitBits0 - e) : 0.0;
      w.next();
    }
  } else {
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = 0.0;
  }
  write_slot<S>(x, planes, (o.rows + 31) / 32, kp / 32, g, kq >> 1, rr + 32 * (int)(kq & 1));
}

// The same for operands whose contraction index is contiguous (s_kc = 1): the 32 rows x 128 k of
// the workgroup are first read along k into LDS (coalesced), then cut slot by slot.  Grid
// (row group, 128 k, z), or with zfast (z, 128 k, row group), as in split_max_kernel.
template <int S>
__global__ void __launch_bounds__(256) split_slice_kmajor_kernel(OpMap o, int64_t K, int64_t kp, int64_t y0,
                                                                 int8_t* planes, const int* ex, int64_t ps,
                                                                 int64_t exs, int zfast) {
  __shared__ double tile[32][129];
  const int64_t z = zfast ? blockIdx.x : blockIdx.z;
  o.p += z * o.s_z;
  planes += z * ps;
  ex += z * exs;
  const int t = threadIdx.x;
  const int64_t g = zfast ? blockIdx.z : blockIdx.x, k0 = (y0 + blockIdx.y) * 128;
  {
    // element (32 g + (t >> 7) + 2 j, k0 + (t & 127)): one column k per thread
    const int64_t k = k0 + (t & 127);
    const int64_t koff = k < K ? (k / o.kc_n) * o.s_kb + (k % o.kc_n) * o.s_kc : 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int rr = (t >> 7) + 2 * j;
      const int64_t r = 32 * g + rr;
      tile[rr][t & 127] = r < o.rows && k < K ? opmap_row(o, r)[koff] : 0.0;
    }
  }
  __syncthreads();
  const int rr = t & 31, kq = t >> 5;
  const int64_t r = 32 * g + rr, kq16 = k0 / 16 + kq;
  if (16 * kq16 >= kp) return;
  const int e = r < o.rows ? ex[r] : 0;
  double x[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) x[q] = ldexp(tile[rr][16 * kq + q], kSplitBits0 - e);
  write_slot<S>(x, planes, (o.rows + 31) / 32, kp / 32, g, kq16 >> 1, rr + 32 * (int)(kq16 & 1));
}

// Row r = (P, m) of the unpacked b^P (element k = b^P_{mk}, packed at T(max) + min), one
// workgroup per row of rpad32(naux * nao); rows past naux * nao are zero.
template <int S>
__global__ void __launch_bounds__(256) split_packed_kernel(const double* __restrict__ B, int64_t nao, int64_t npair,
                                                           int64_t kp, int8_t* planes, int* ex, int64_t rows) {
  const int64_t r = blockIdx.x;
  const int t = threadIdx.x;
  const int64_t G = (rows + 31) / 32, KB = kp / 32, g = r / 32;
  const int rr = (int)(r % 32);
  if (r >= rows) {
    double z[16];
    for (int64_t kq = t; kq < kp / 16; kq += 256) {
#pragma unroll
      for (int q = 0; q < 16; ++q) z[q] = 0.0;
      write_slot<S>(z, planes, G, KB, g, kq >> 1, rr + 32 * (int)(kq & 1));
    }
    return;
  }
  const int64_t P = r / nao, m = r % nao;
  const double* Bp = B + P * npair;
  auto elem = [&](int64_t k) {
    const int64_t hi = m > k ? m : k, lo = m > k ? k : m;
    return Bp[hi * (hi + 1) / 2 + lo];
  };
  double mx = 0.0;
  for (int64_t k = t; k < nao; k += 256) mx = fmax(mx, fabs(elem(k)));
  const int e = row_exponent(block_max(mx));
  if (t == 0) ex[r] = e;
  double x[16];
  for (int64_t kq = t; kq < kp / 16; kq += 256) {
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = 16 * kq + q < nao ? ldexp(elem(16 * kq + q), kSplitBits0 - e) : 0.0;
    write_slot<S>(x, planes, G, KB, g, kq >> 1, rr + 32 * (int)(kq & 1));
  }
}

// Rows mu of the DF tensor over k = (P, nu), k = P nao + nu (element b^P_{mu nu}): the operand
// of products that contract over (P, nu).  Exponent of row mu: the largest row exponent over
// P, taken per (P, mu) row with one workgroup each and merged by integer atomic max.
__global__ void __launch_bounds__(256) split_packed_t_max_kernel(const double* __restrict__ B, int64_t nao,
                                                                 int64_t npair, int* ex) {
  const int64_t r = blockIdx.x, P = r / nao, m = r % nao;
  const double* Bp = B + P * npair;
  double mx = 0.0;
  for (int64_t k = threadIdx.x; k < nao; k += 256) {
    const int64_t hi = m > k ? m : k, lo = m > k ? k : m;
    mx = fmax(mx, fabs(Bp[hi * (hi + 1) / 2 + lo]));
  }
  mx = block_max(mx);
  if (threadIdx.x == 0 && mx > 0.0) atomicMax(ex + m, row_exponent(mx));
}

// One workgroup per (row group g = blockIdx.x, 128 k); thread t fills slot (rr = t % 32, 16 k at
// 16 (t / 32)) of its block in every plane.  Lanes run along mu: for mu <= nu the 32 elements
// of a load are one run of packed row nu.
template <int S>
__global__ void __launch_bounds__(256) split_packed_t_kernel(const double* __restrict__ B, int64_t naux,
                                                             int64_t nao, int64_t npair, int64_t kp, int64_t y0,
                                                             int8_t* planes, const int* ex) {
  const int t = threadIdx.x, rr = t & 31;
  const int64_t g = blockIdx.x, kq = (y0 + blockIdx.y) * 8 + (t >> 5);
  if (16 * kq >= kp) return;
  const int64_t m = 32 * g + rr, K = naux * nao;
  double x[16];
  if (m < nao) {
    const int e = ex[m];
    int64_t k = 16 * kq, P = k / nao, nu = k % nao;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      double v = 0.0;
      if (k + q < K) {
        const int64_t hi = m > nu ? m : nu, lo = m > nu ? nu : m;
        v = B[P * npair + hi * (hi + 1) / 2 + lo];
      }
      x[q] = ldexp(v, kSplitBits0 - e);
      if (++nu == nao) {
        nu = 0;
        ++P;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = 0.0;
  }
  write_slot<S>(x, planes, (nao + 31) / 32, kp / 32, g, kq >> 1, rr + 32 * (int)(kq & 1));
}

// ---------------------------------------------------------------------------------------
// Slice product.  Workgroup tile 64 x 64 over 4 waves (2 x 2) of 32 x 32, one
// v_mfma_i32_32x32x32_i8 per slice pair and 32-deep k step.  Each k step moves S (2 + 2) blocks
// of 1 KB from HBM / L2 straight into LDS (global_load_lds, no staging registers), two LDS
// stages deep (56 KB at S = 7); a wave reads its S + S operand fragments as one 16-byte LDS read
// per lane each.  One int32 accumulator per slice diagonal d = s + t (exact over kMaxSteps steps =
// 32768 k, so every split is at most that long and no FP64 sums are kept in the loop).  About 170
// registers per lane.  Two workgroups share each CU (two waves per SIMD from different
// workgroups), so one workgroup's barrier and load waits hide behind the other's MFMAs; a single
// workgroup of 8 waves on 128 x 64 tiles with three stages, every wave at the same barrier, took
// 66.2 ms for the paper-scale half transform against 62.9 ms.  With `tri` (M == N), tiles wholly
// above the diagonal exit.
constexpr int kGM = 64, kGN = 64, kKS = 32, kStages = 2, kWaves = 4;
constexpr int kMaxSteps = 1024;

template <int S>
struct SliceTile {
  static constexpr int GA = kGM / 32, GB = kGN / 32;
  static constexpr int NBLK = S * (GA + GB);        // blocks per k step
  static constexpr int STAGE = NBLK * 1024;
  static constexpr int LPW = (NBLK + kWaves - 1) / kWaves;   // direct loads per wave and step (at most)
  static constexpr int LPW_MIN = NBLK / kWaves;               // ... and at least
};

typedef __attribute__((address_space(3))) void* lds_ptr_t;

template <int S, bool GEN>
__global__ void __launch_bounds__(64 * kWaves, 2) slice_gemm_kernel(const int8_t* __restrict__ Ap, const int* __restrict__ ea,
                                                            int64_t M, const int8_t* __restrict__ Bp,
                                                            const int* __restrict__ eb, int64_t N, int64_t KB,
                                                            OutMap O, int64_t tilesM, int64_t tilesN, int tri,
                                                            double* part, SliceBatch zs) {
  typedef SliceTile<S> T;
  __shared__ __attribute__((aligned(1024))) int8_t lds[kStages * T::STAGE];
  // product z of a batch (grid z): its operands and outputs at the batch strides
  const int64_t z = blockIdx.z, nz = gridDim.z;
  Ap += z * zs.a;
  ea += z * zs.ea;
  Bp += z * zs.b;
  eb += z * zs.eb;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % (kGM / 32), wn = wave / (kGM / 32);
  // (tile, split) of this workgroup.  With the split count a multiple of 8, whole splits are dealt
  // to the XCDs (workgroup L of the dispatch order runs on XCD L % 8): XCD x runs splits x, x + 8,
  // ... each with all its tiles side by side, which stream the same operand rows of one k range
  // through that XCD's L2 at about the same time.  Otherwise the tiles of each split are grouped
  // per XCD.  Both are bijections of [0, tiles x nsplit).
  const int nsplit = gridDim.y;
  const int64_t ntile = tilesM * tilesN;
  int split;
  int64_t tile;
  if (nsplit >= 8 && nsplit % 8 == 0) {
    const int64_t L = blockIdx.x + (int64_t)gridDim.x * blockIdx.y, j = L / 8;
    split = (int)(L % 8 + 8 * (j / ntile));
    tile = j % ntile;
  } else {
    split = blockIdx.y;
    tile = xcd_remap_i8(blockIdx.x, ntile);
  }
  const int64_t I = tile / tilesN, J = tile % tilesN;   // column tiles of one row band side by side
  if (tri && J * kGN > I * kGM + kGM - 1) return;       // no element on or below the diagonal
  const int64_t GAn = (M + 31) / 32, GBn = (N + 31) / 32;
  const int64_t ks0 = KB * split / nsplit, ks1 = KB * (split + 1) / nsplit;

  // this wave's direct loads: blocks j = wave + kWaves i of the step (A blocks s * GA + g first)
  const int8_t* gp[T::LPW];
  int loff[T::LPW];
#pragma unroll
  for (int i = 0; i < T::LPW; ++i) {
    int j = wave + kWaves * i;
    if (j >= T::NBLK) j = T::NBLK - 1;   // unused slot (never issued)
    loff[i] = j * 1024;
    if (j < S * T::GA) {
      const int s = j / T::GA;
      int64_t g = I * T::GA + j % T::GA;
      if (g >= GAn) g = GAn - 1;         // past the last row group: its outputs are not stored
      gp[i] = Ap + block_offset(s, g, 0, GAn, KB) + 16 * lane;
    } else {
      const int s = (j - S * T::GA) / T::GB;
      int64_t g = J * T::GB + (j - S * T::GA) % T::GB;
      if (g >= GBn) g = GBn - 1;
      gp[i] = Bp + block_offset(s, g, 0, GBn, KB) + 16 * lane;
    }
  }
  auto issue = [&](int st, int64_t ks) {
#pragma unroll
    for (int i = 0; i < T::LPW; ++i)
      if (i < T::LPW_MIN || wave + kWaves * i < T::NBLK)
        __builtin_amdgcn_global_load_lds((const void*)(gp[i] + ks * 1024), (lds_ptr_t)(lds + st * T::STAGE + loff[i]),
                                         16, 0, 0);
  };

  v16i acc[S];
#pragma unroll
  for (int d = 0; d < S; ++d)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[d][e] = 0;

  // a wave whose 32 rows or 32 columns all lie past the end only takes part in loads and barriers
  const bool live = I * kGM + 32 * wm < M && J * kGN + 32 * wn < N;
  const int8_t* fa0 = lds + wm * 1024 + 16 * lane;
  const int8_t* fb0 = lds + (S * T::GA + wn) * 1024 + 16 * lane;
#pragma unroll
  for (int p = 0; p < kStages - 1; ++p)
    if (ks0 + p < ks1) issue(p, ks0 + p);
  int st = 0;
  for (int64_t ks = ks0; ks < ks1; ++ks) {
    // this wave's loads of step ks have landed once at most the later steps' are outstanding
    // (with two stages none are: step ks + 1 is issued after this barrier)
    constexpr int kLater = T::LPW_MIN * (kStages > 2 ? kStages - 2 : 0);
    if (kLater > 0 && ks + 1 < ks1) __builtin_amdgcn_s_waitcnt(kVmcnt<kLater>::imm);
    else __builtin_amdgcn_s_waitcnt(kVmcnt<0>::imm);
    // every wave's loads of step ks are in LDS, and its reads of step ks - 1 (into the stage the
    // next issue overwrites) are done.  A plain barrier: a workgroup fence would also wait for
    // the loads of step ks + 1.
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (ks + kStages - 1 < ks1) issue(st == 0 ? kStages - 1 : st - 1, ks + kStages - 1);
    if (!live) {
      st = st == kStages - 1 ? 0 : st + 1;
      continue;
    }
    v4i fa[S], fb[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      fa[s] = *(const v4i*)(fa0 + st * T::STAGE + s * T::GA * 1024);
      fb[s] = *(const v4i*)(fb0 + st * T::STAGE + s * T::GB * 1024);
    }
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int u = 0; u + s < S; ++u) acc[s + u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[s], fb[u], acc[s + u], 0, 0, 0);
    st = st == kStages - 1 ? 0 : st + 1;
  }

  // epilogue: value = 2^(ea + eb - 12) sum_d 2^(-7 d) I_d.  D[i][j] of the 32 x 32 tile is in
  // lane j + 32 ((i / 4) % 2), element 4 (i / 8) + i % 4.
  const int64_t m0 = I * kGM + 32 * wm, n = J * kGN + 32 * wn + (lane & 31);
  if (n >= N) return;
  const int ebn = eb[n];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int64_t m = m0 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
    if (m >= M) continue;
    double F = 0.0;
#pragma unroll
    for (int d = S - 1; d >= 0; --d) F += ldexp((double)acc[d][e], -kSplitBits * d);
    const double val = ldexp(F, ea[m] + ebn - 2 * kSplitBits0);
    if (part) {
      part[(((int64_t)split * nz + z) * M + m) * N + n] = val;
    } else {
      double* dst;
      if (n < O.nsplit) {
        const int64_t nh = O.s_nh ? n / O.nl : 0, mh = O.s_mh ? m / O.ml : 0;
        dst = O.p + z * O.s_z + (mh * O.s_mh + (m - mh * O.ml) * O.s_ml) + (nh * O.s_nh + (n - nh * O.nl) * O.s_nl);
      } else {
        dst = O.p2 + z * O.s2_z + m * O.s2_m + (n - O.nsplit);
      }
      if (GEN) *dst = O.accumulate ? *dst + O.alpha * val : O.alpha * val;
      else *dst = val;
    }
  }
}

}  // namespace

int64_t kpad64(int64_t n) { return (n + 63) / 64 * 64; }
int64_t rpad32(int64_t n) { return (n + 31) / 32 * 32; }
int64_t split_plane_bytes(int64_t rows, int64_t K, int nslice) { return (int64_t)nslice * rpad32(rows) * kpad64(K); }

template <int S>
static hipError_t split_rows_s(const OpMap& o, int64_t K, int8_t* planes, int* ex, int64_t nz, int64_t ps,
                               int64_t exs, hipStream_t s) {
  const int64_t kp = kpad64(K);
  const unsigned ng = (unsigned)(rpad32(o.rows) / 32), z = (unsigned)nz;
  // rows adjacent in memory with the contraction index elsewhere: lanes along the rows
  const bool rows_adjacent = o.s_rlo == 1 && o.s_kc != 1;
  if (exs == o.rows || nz == 1) {
    fill_int_kernel<<<(unsigned)((o.rows * nz + 255) / 256), 256, 0, s>>>(ex, o.rows * nz, kNoExponent);
  } else {
    for (int64_t i = 0; i < nz; ++i)
      fill_int_kernel<<<(unsigned)((o.rows + 255) / 256), 256, 0, s>>>(ex + i * exs, o.rows, kNoExponent);
  }
  if (rows_adjacent) {
    const int64_t ny = (K + kSplitChunkR - 1) / kSplitChunkR;
    for (int64_t y0 = 0; y0 < ny; y0 += 65535) {
      const unsigned n = (unsigned)(ny - y0 < 65535 ? ny - y0 : 65535);
      split_max_rows_kernel<<<dim3(ng, n, z), 256, 0, s>>>(o, K, y0, ex, exs);
    }
  } else {
    const int64_t nc = (K + kSplitChunk - 1) / kSplitChunk;
    const bool zfast = nz > 1 && nc <= 65535;
    for (int64_t r0 = 0; r0 < o.rows; r0 += 65535) {   // grid y carries the row
      const unsigned nr = (unsigned)(o.rows - r0 < 65535 ? o.rows - r0 : 65535);
      const dim3 grid = zfast ? dim3(z, nr, (unsigned)nc) : dim3((unsigned)nc, nr, z);
      split_max_kernel<<<grid, 256, 0, s>>>(o, K, r0, ex, exs, zfast ? 1 : 0);
    }
  }
  const int64_t ny = (kp + 127) / 128;   // grid y carries 128 k
  const bool zfast = nz > 1 && ng <= 65535;
  for (int64_t y0 = 0; y0 < ny; y0 += 65535) {
    const unsigned n = (unsigned)(ny - y0 < 65535 ? ny - y0 : 65535);
    if (o.s_kc == 1)
      split_slice_kmajor_kernel<S><<<zfast ? dim3(z, n, ng) : dim3(ng, n, z), 256, 0, s>>>(o, K, kp, y0, planes, ex,
                                                                                          ps, exs, zfast ? 1 : 0);
    else split_slice_kernel<S><<<dim3(ng, n, z), 256, 0, s>>>(o, K, kp, y0, planes, ex, ps, exs);
  }
  return hipGetLastError();
}

hipError_t launch_split_rows_batched(const OpMap& o, int64_t K, int nslice, int8_t* planes, int* ex, int64_t nz,
                                     int64_t plane_stride, int64_t ex_stride, hipStream_t s) {
  if (o.rows <= 0 || nz == 0) return hipSuccess;
  if (rpad32(o.rows) > 0x7fffffffLL || K <= 0 || (K + kSplitChunk - 1) / kSplitChunk > 0x7fffffffLL || nz < 0 ||
      nz > 65535 || (nz > 1 && ex_stride < o.rows))
    return hipErrorInvalidValue;
  switch (nslice) {
    case 4: return split_rows_s<4>(o, K, planes, ex, nz, plane_stride, ex_stride, s);
    case 5: return split_rows_s<5>(o, K, planes, ex, nz, plane_stride, ex_stride, s);
    case 6: return split_rows_s<6>(o, K, planes, ex, nz, plane_stride, ex_stride, s);
    case 7: return split_rows_s<7>(o, K, planes, ex, nz, plane_stride, ex_stride, s);
    case 8: return split_rows_s<8>(o, K, planes, ex, nz, plane_stride, ex_stride, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_split_rows(const OpMap& o, int64_t K, int nslice, int8_t* planes, int* ex, hipStream_t s) {
  OpMap o1 = o;
  o1.s_z = 0;
  return launch_split_rows_batched(o1, K, nslice, planes, ex, 1, 0, 0, s);
}

template <int S>
static hipError_t split_packed_s(const double* B, int64_t naux, int64_t nao, int8_t* planes, int* ex,
                                 hipStream_t s) {
  const int64_t rows = naux * nao;
  split_packed_kernel<S><<<(unsigned)rpad32(rows), 256, 0, s>>>(B, nao, nao * (nao + 1) / 2, kpad64(nao), planes, ex,
                                                                rows);
  return hipGetLastError();
}

hipError_t launch_split_packed(const double* B, int64_t naux, int64_t nao, int nslice, int8_t* planes, int* ex,
                               hipStream_t s) {
  const int64_t rows = naux * nao;
  if (rows <= 0) return hipSuccess;
  if (rpad32(rows) > 0x7fffffffLL) return hipErrorInvalidValue;
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
static hipError_t split_packed_t_s(const double* B, int64_t naux, int64_t nao, int8_t* planes, int* ex,
                                   hipStream_t s) {
  const int64_t npair = nao * (nao + 1) / 2, kp = kpad64(naux * nao);
  fill_int_kernel<<<(unsigned)((nao + 255) / 256), 256, 0, s>>>(ex, nao, kNoExponent);
  split_packed_t_max_kernel<<<(unsigned)(naux * nao), 256, 0, s>>>(B, nao, npair, ex);
  const int64_t ny = (kp + 127) / 128;
  for (int64_t y0 = 0; y0 < ny; y0 += 65535) {
    const unsigned n = (unsigned)(ny - y0 < 65535 ? ny - y0 : 65535);
    split_packed_t_kernel<S><<<dim3((unsigned)(rpad32(nao) / 32), n), 256, 0, s>>>(B, naux, nao, npair, kp, y0,
                                                                                   planes, ex);
  }
  return hipGetLastError();
}

hipError_t launch_split_packed_t(const double* B, int64_t naux, int64_t nao, int nslice, int8_t* planes, int* ex,
                                 hipStream_t s) {
  if (naux <= 0 || nao <= 0) return hipSuccess;
  if (naux * nao > 0x7fffffffLL) return hipErrorInvalidValue;
  switch (nslice) {
    case 4: return split_packed_t_s<4>(B, naux, nao, planes, ex, s);
    case 5: return split_packed_t_s<5>(B, naux, nao, planes, ex, s);
    case 6: return split_packed_t_s<6>(B, naux, nao, planes, ex, s);
    case 7: return split_packed_t_s<7>(B, naux, nao, planes, ex, s);
    case 8: return split_packed_t_s<8>(B, naux, nao, planes, ex, s);
    default: return hipErrorInvalidValue;
  }
}

static int64_t slice_tiles_m(int64_t M) { return (M + kGM - 1) / kGM; }
static int64_t slice_tiles_n(int64_t N) { return (N + kGN - 1) / kGN; }

int64_t slice_gemm_tiles(int64_t M, int64_t N, bool tri) {
  const int64_t tm = slice_tiles_m(M), tn = slice_tiles_n(N);
  if (!tri) return tm * tn;
  int64_t c = 0;
  for (int64_t I = 0; I < tm; ++I) {
    const int64_t jmax = (I * kGM + kGM - 1) / kGN + 1;
    c += jmax < tn ? jmax : tn;
  }
  return c;
}
int64_t slice_gemm_steps(int64_t kp) { return kp / kKS; }
int64_t slice_gemm_max_steps() { return kMaxSteps; }

template <int S>
static void slice_gemm_s(const int8_t* A, const int* ea, int64_t M, const int8_t* B, const int* eb, int64_t N,
                         int64_t kp, const OutMap& O, bool tri, int nsplit, double* part, int64_t nz,
                         const SliceBatch& zs, hipStream_t s) {
  const int64_t tm = slice_tiles_m(M), tn = slice_tiles_n(N);
  const dim3 grid((unsigned)(tm * tn), (unsigned)nsplit, (unsigned)nz);
  const bool gen = !part && (O.alpha != 1.0 || O.accumulate);
  if (gen) slice_gemm_kernel<S, true><<<grid, 64 * kWaves, 0, s>>>(A, ea, M, B, eb, N, kp / kKS, O, tm, tn, tri, part, zs);
  else slice_gemm_kernel<S, false><<<grid, 64 * kWaves, 0, s>>>(A, ea, M, B, eb, N, kp / kKS, O, tm, tn, tri, part, zs);
}

hipError_t launch_slice_gemm(const int8_t* A, const int* ea, int64_t M, const int8_t* B, const int* eb, int64_t N,
                             int64_t kp, int nslice, const OutMap& O, bool tri, int nsplit, double* part,
                             hipStream_t s) {
  return launch_slice_gemm_batched(A, ea, M, B, eb, N, kp, nslice, O, tri, nsplit, part, 1, SliceBatch{}, s);
}

hipError_t launch_slice_gemm_batched(const int8_t* A, const int* ea, int64_t M, const int8_t* B, const int* eb,
                                     int64_t N, int64_t kp, int nslice, const OutMap& O, bool tri, int nsplit,
                                     double* part, int64_t nz, const SliceBatch& zs, hipStream_t s) {
  if (M <= 0 || N <= 0 || nz == 0) return hipSuccess;
  if (kp % 64 != 0 || kp <= 0 || nsplit < 1 || nsplit > 65535 || (tri && M != N) || (nsplit > 1 && !part) ||
      nz < 0 || nz > 65535)
    return hipErrorInvalidValue;
  // every split at most kMaxSteps steps long: the int32 diagonal sums stay exact
  if ((kp / kKS + nsplit - 1) / nsplit > kMaxSteps) return hipErrorInvalidValue;
  if (slice_tiles_m(M) * slice_tiles_n(N) > 0x7fffffffLL) return hipErrorInvalidValue;
  switch (nslice) {
    case 4: slice_gemm_s<4>(A, ea, M, B, eb, N, kp, O, tri, nsplit, part, nz, zs, s); break;
    case 5: slice_gemm_s<5>(A, ea, M, B, eb, N, kp, O, tri, nsplit, part, nz, zs, s); break;
    case 6: slice_gemm_s<6>(A, ea, M, B, eb, N, kp, O, tri, nsplit, part, nz, zs, s); break;
    case 7: slice_gemm_s<7>(A, ea, M, B, eb, N, kp, O, tri, nsplit, part, nz, zs, s); break;
    case 8: slice_gemm_s<8>(A, ea, M, B, eb, N, kp, O, tri, nsplit, part, nz, zs, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace dfk
