// HIP kernels for gfx950 (MI355X): FP64 contractions of the packed Cholesky tensor.
//
// Every dense contraction runs on the FP64 matrix cores (v_mfma_f64_16x16x4_f64,
// 64 cycles per issue per SIMD).  Operand tiles are staged through LDS in a
// [row][k] layout with a row stride of 17 doubles: both the "k fastest" and the
// "row fastest" global-load mappings then write, and the MFMA operand reads
// then read, 32 lanes per LDS cycle without bank conflicts.
//
// Operand layout of v_mfma_f64_16x16x4_f64 (measured on gfx950):
//   A[i][k] in lane i + 16k, B[k][j] in lane j + 16k,
//   D[i][j] in lane j + 16*(i%4), accumulator register i/4.
#include "kernels.h"

#include <math.h>

namespace dfk {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int WM_, int WN_, int TM_, int TN_>
struct Cfg {
  static constexpr int WM = WM_, WN = WN_, TM = TM_, TN = TN_;
  static constexpr int NT = 64 * WM * WN;
  static constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN, BK = 16;
  static constexpr int LD = BK + 1;
  static constexpr int LDS_A = BM * LD, LDS_B = BN * LD;
  static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "tile must split evenly over threads");
};

// 128 x 128 output tile, 4 waves of 64 x 64 (4 x 4 MFMA blocks each).
typedef Cfg<2, 2, 4, 4> CfgBig;

// ---------------------------------------------------------------------------------------
// Block index -> work item, keeping runs of consecutive work items on one XCD.  The
// dispatcher hands consecutive workgroups to the 8 XCDs in turn; this remap makes XCD x
// process the x-th eighth of the index range in order, so tiles that share operands
// (the same P slab, the same B tile) share that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t id, int64_t n) {
  const int64_t full = (n / 8) * 8;
  if (id >= full) return id;
  return (id % 8) * (full / 8) + id / 8;
}

template <class C>
__device__ __forceinline__ void mma_slab(const double* __restrict__ As, const double* __restrict__ Bs,
                                         d4 (&acc)[C::TM][C::TN], int wm, int wn, int lane) {
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < C::BK; kk += 4) {
    double a[C::TM], b[C::TN];
#pragma unroll
    for (int i = 0; i < C::TM; ++i) a[i] = As[((wm * C::TM + i) * 16 + lr) * C::LD + kk + lk];
#pragma unroll
    for (int j = 0; j < C::TN; ++j) b[j] = Bs[((wn * C::TN + j) * 16 + lr) * C::LD + kk + lk];
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

template <class C>
__device__ __forceinline__ void zero_acc(d4 (&acc)[C::TM][C::TN]) {
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
}

template <class C>
__device__ __forceinline__ void store_tile(const OutMap& o, int64_t z, int64_t m0, int64_t n0,
                                           const d4 (&acc)[C::TM][C::TN], int wm, int wn, int lane) {
  const int lr = lane & 15, lg = lane >> 4;
  double* base = o.p + z * o.s_z;
#pragma unroll
  for (int j = 0; j < C::TN; ++j) {
    const int64_t n = n0 + (wn * C::TN + j) * 16 + lr;
    if (n >= o.N) continue;
    const int64_t noff = (n / o.nl) * o.s_nh + (n % o.nl) * o.s_nl;
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + (wm * C::TM + i) * 16 + 4 * r + lg;
        if (m < o.M) base[(m / o.ml) * o.s_mh + (m % o.ml) * o.s_ml + noff] = acc[i][j][r];
      }
  }
}

// Global -> register -> LDS loader for one operand described by an OpMap.
//   KC = true : lanes run along k (16 consecutive k of one row per 16 lanes)
//   KC = false: lanes run along the row index
template <class C, int R, bool KC>
struct Loader {
  static constexpr int E = R * C::BK / C::NT;
  int64_t off[E];
  bool ok[E];
  int64_t kso;

  __device__ __forceinline__ static int rr(int t, int q) {
    const int e = t + C::NT * q;
    return KC ? e / C::BK : e % R;
  }
  __device__ __forceinline__ static int kk(int t, int q) {
    const int e = t + C::NT * q;
    return KC ? e % C::BK : e / R;
  }
  __device__ __forceinline__ void init(const OpMap& o, int64_t r0, int64_t z, int t) {
    kso = z * o.s_ksz;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int64_t r = r0 + rr(t, q);
      ok[q] = r < o.rows;
      off[q] = ok[q] ? z * o.s_z + (r / o.rl) * o.s_rh + (r % o.rl) * o.s_rlo : 0;
    }
  }
  __device__ __forceinline__ void load(const OpMap& o, int64_t kb, int64_t kc0, int t, double (&v)[E]) const {
    const int64_t kbo = kb * o.s_kb;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int64_t kc = kc0 + kk(t, q);
      v[q] = (ok[q] && kc < o.kc_n) ? o.p[off[q] + kbo + kc * o.s_kc] : 0.0;
      if (o.ks && kc < o.kc_n) v[q] *= o.ks[kso + kc];
    }
  }
  __device__ __forceinline__ static void store(double* S, int t, const double (&v)[E]) {
#pragma unroll
    for (int q = 0; q < E; ++q) S[rr(t, q) * C::LD + kk(t, q)] = v[q];
  }
};

// ---------------------------------------------------------------------------------------
// Generic tiled product  C(m, n) = sum_k A(m, k) B(n, k)  over a batch (grid z).
template <class C, bool AK, bool BK>
__global__ void __launch_bounds__(C::NT) gemm_kernel(OpMap A, OpMap B, OutMap O, int64_t tilesM,
                                                     int64_t tilesN) {
  __shared__ double smem[2 * (C::LDS_A + C::LDS_B)];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave % C::WM, wn = wave / C::WM;
  const int64_t ntile = tilesM * tilesN;
  const int64_t tile = xcd_remap(blockIdx.x, ntile);
  const int64_t z = blockIdx.z;
  const int64_t m0 = (tile % tilesM) * C::BM, n0 = (tile / tilesM) * C::BN;

  Loader<C, C::BM, AK> la;
  Loader<C, C::BN, BK> lb;
  la.init(A, m0, z, t);
  lb.init(B, n0, z, t);
  constexpr int STAGE = C::LDS_A + C::LDS_B;
#define As(b) (smem + (b) * STAGE)
#define Bs(b) (smem + (b) * STAGE + C::LDS_A)

  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  const int64_t nkc = (A.kc_n + C::BK - 1) / C::BK;
  const int64_t nslab = A.kb_n * nkc;
  double va[Loader<C, C::BM, AK>::E], vb[Loader<C, C::BN, BK>::E];
  if (nslab > 0) {
    la.load(A, 0, 0, t, va);
    lb.load(B, 0, 0, t, vb);
    la.store(As(0), t, va);
    lb.store(Bs(0), t, vb);
  }
  __syncthreads();
  int64_t kb = 0, kc0 = 0;
  for (int64_t s = 0; s < nslab; ++s) {
    const int cur = s & 1;
    const bool more = s + 1 < nslab;
    if (more) {
      kc0 += C::BK;
      if (kc0 >= A.kc_n) { kc0 = 0; ++kb; }
      la.load(A, kb, kc0, t, va);
      lb.load(B, kb, kc0, t, vb);
    }
    mma_slab<C>(As(cur), Bs(cur), acc, wm, wn, lane);
    if (more) {
      la.store(As(cur ^ 1), t, va);
      lb.store(Bs(cur ^ 1), t, vb);
    }
    __syncthreads();
  }
  store_tile<C>(O, z, m0, n0, acc, wm, wn, lane);
}

// ---------------------------------------------------------------------------------------
// Lower-triangle tile SYRK with the kb range split over workgroups:
// Kpart[split][z] tile (I, J), I >= J, = sum_{kb in split} sum_kc A(i, kb, kc) A(j, kb, kc).
template <class C>
__global__ void __launch_bounds__(C::NT) syrk_kernel(OpMap A, OpMap Bw, int64_t n, int64_t nz, int nsplit,
                                                     int64_t npairs, double* Kpart) {
  static_assert(C::BM == C::BN, "square tiles");
  __shared__ double smem[2 * (C::LDS_A + C::LDS_B)];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave % C::WM, wn = wave / C::WM;
  const int64_t nitem = npairs * nsplit;
  const int64_t item = xcd_remap(blockIdx.x, nitem);
  const int64_t z = blockIdx.z;
  const int64_t pair = item % npairs;
  const int split = (int)(item / npairs);
  // triangular decode: pair = I(I+1)/2 + J, 0 <= J <= I
  int64_t I = (int64_t)((sqrt(8.0 * (double)pair + 1.0) - 1.0) * 0.5);
  while (I * (I + 1) / 2 > pair) --I;
  while ((I + 1) * (I + 2) / 2 <= pair) ++I;
  const int64_t J = pair - I * (I + 1) / 2;
  const int64_t m0 = I * C::BM, n0 = J * C::BN;
  const int64_t kb_lo = A.kb_n * split / nsplit, kb_hi = A.kb_n * (split + 1) / nsplit;

  Loader<C, C::BM, true> la;
  Loader<C, C::BN, true> lb;
  la.init(A, m0, z, t);
  lb.init(Bw, n0, z, t);
  constexpr int STAGE = C::LDS_A + C::LDS_B;
#define As(b) (smem + (b) * STAGE)
#define Bs(b) (smem + (b) * STAGE + C::LDS_A)

  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  const int64_t nkc = (A.kc_n + C::BK - 1) / C::BK;
  const int64_t nslab = (kb_hi - kb_lo) * nkc;
  double va[Loader<C, C::BM, true>::E], vb[Loader<C, C::BN, true>::E];
  if (nslab > 0) {
    la.load(A, kb_lo, 0, t, va);
    lb.load(Bw, kb_lo, 0, t, vb);
    la.store(As(0), t, va);
    lb.store(Bs(0), t, vb);
  }
  __syncthreads();
  int64_t kb = kb_lo, kc0 = 0;
  for (int64_t s = 0; s < nslab; ++s) {
    const int cur = s & 1;
    const bool more = s + 1 < nslab;
    if (more) {
      kc0 += C::BK;
      if (kc0 >= A.kc_n) { kc0 = 0; ++kb; }
      la.load(A, kb, kc0, t, va);
      lb.load(Bw, kb, kc0, t, vb);
    }
    mma_slab<C>(As(cur), Bs(cur), acc, wm, wn, lane);
    if (more) {
      la.store(As(cur ^ 1), t, va);
      lb.store(Bs(cur ^ 1), t, vb);
    }
    __syncthreads();
  }
  OutMap o = out_plain(Kpart + ((int64_t)split * nz + z) * n * n, n, n, n);
  o.s_z = 0;
  store_tile<C>(o, 0, m0, n0, acc, wm, wn, lane);
}

__global__ void __launch_bounds__(256) syrk_reduce_kernel(const double* __restrict__ Kpart, int nsplit,
                                                          int64_t n, int64_t nz, double* __restrict__ K) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nn = n * n;
  if (idx >= nn * nz) return;
  const int64_t z = idx / nn, rem = idx % nn, i = rem / n, j = rem % n;
  const int64_t a = i >= j ? i : j, b = i >= j ? j : i;   // the lower element, computed by the SYRK tiles
  double s = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) s += Kpart[((int64_t)sp * nz + z) * nn + a * n + b];
  K[idx] = s;
}

// ---------------------------------------------------------------------------------------
// Half transform of one packed, symmetric b^P against a dense C.
// A operand element (m, k) = b^P_{mk}: a tile strictly below the diagonal is read along k
// (contiguous runs of a packed row), a tile strictly above it along m (contiguous runs of
// packed row k), a tile on the diagonal element by element through max/min.
template <class C>
__global__ void __launch_bounds__(C::NT) half_kernel(const double* __restrict__ B, int64_t naux, int nao,
                                                     int64_t npair, OpMap Cm, double* __restrict__ X,
                                                     int64_t ldx, int64_t tilesM, int64_t tilesN) {
  __shared__ double smem[2 * (C::LDS_A + C::LDS_B)];
  constexpr int EA = C::BM * C::BK / C::NT;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave % C::WM, wn = wave / C::WM;
  const int64_t ntile = tilesM * tilesN;
  const int64_t item = xcd_remap(blockIdx.x, ntile * naux);
  const int64_t P = item / ntile, tile = item % ntile;
  const int m0 = (int)((tile % tilesM) * C::BM), n0 = (int)((tile / tilesM) * C::BN);
  const double* __restrict__ Bp = B + P * npair;

  Loader<C, C::BN, false> lb;
  lb.init(Cm, n0, 0, t);
  constexpr int STAGE = C::LDS_A + C::LDS_B;
#define As(b) (smem + (b) * STAGE)
#define Bs(b) (smem + (b) * STAGE + C::LDS_A)

  // A tile loader: returns values and their LDS slots for slab k0
  auto load_a = [&](int k0, double (&v)[EA], int (&slot)[EA]) {
    const bool below = k0 + C::BK - 1 <= m0;
    const bool above = k0 >= m0 + C::BM - 1;
#pragma unroll
    for (int q = 0; q < EA; ++q) {
      const int e = t + C::NT * q;
      if (below) {
        const int r = e / C::BK, k = e % C::BK;
        const int m = m0 + r, kg = k0 + k;
        v[q] = m < nao ? Bp[(int64_t)m * (m + 1) / 2 + kg] : 0.0;
        slot[q] = r * C::LD + k;
      } else {
        const int r = e % C::BM, k = e / C::BM;
        const int m = m0 + r, kg = k0 + k;
        if (above) {
          v[q] = kg < nao ? Bp[(int64_t)kg * (kg + 1) / 2 + m] : 0.0;
        } else {
          const int hi = m > kg ? m : kg, lo = m > kg ? kg : m;
          v[q] = (m < nao && kg < nao) ? Bp[(int64_t)hi * (hi + 1) / 2 + lo] : 0.0;
        }
        slot[q] = r * C::LD + k;
      }
    }
  };

  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  const int nslab = (nao + C::BK - 1) / C::BK;
  double va[EA], vb[Loader<C, C::BN, false>::E];
  int sa[EA];
  load_a(0, va, sa);
  lb.load(Cm, 0, 0, t, vb);
#pragma unroll
  for (int q = 0; q < EA; ++q) As(0)[sa[q]] = va[q];
  lb.store(Bs(0), t, vb);
  __syncthreads();
  for (int s = 0; s < nslab; ++s) {
    const int cur = s & 1;
    const bool more = s + 1 < nslab;
    if (more) {
      load_a((s + 1) * C::BK, va, sa);
      lb.load(Cm, 0, (int64_t)(s + 1) * C::BK, t, vb);
    }
    mma_slab<C>(As(cur), Bs(cur), acc, wm, wn, lane);
    if (more) {
#pragma unroll
      for (int q = 0; q < EA; ++q) As(cur ^ 1)[sa[q]] = va[q];
      lb.store(Bs(cur ^ 1), t, vb);
    }
    __syncthreads();
  }
  OutMap o = out_plain(X + P * (int64_t)nao * ldx, nao, Cm.rows, ldx);
  store_tile<C>(o, 0, m0, n0, acc, wm, wn, lane);
}

// ---------------------------------------------------------------------------------------
// v[z][P] = sum_{m, c} C[z][m][c] w[z][c] X[P][m][z*nocc + c], one workgroup per (P, z),
// fixed-order reduction (deterministic).
__global__ void __launch_bounds__(256) jvec_kernel(const double* __restrict__ X, int64_t nao, int64_t ldx,
                                                   const double* __restrict__ Cm, const double* __restrict__ w,
                                                   int64_t nocc, double* __restrict__ v, int64_t naux) {
  __shared__ double red[4];
  const int64_t P = blockIdx.x, z = blockIdx.y;
  const double* Xp = X + P * nao * ldx + z * nocc;
  const double* Cz = Cm + z * nao * nocc;
  const double* wz = w ? w + z * nocc : nullptr;
  double s = 0.0;
  int64_t m = threadIdx.x / nocc, c = threadIdx.x % nocc;
  while (m < nao) {
    const double cw = wz ? Cz[m * nocc + c] * wz[c] : Cz[m * nocc + c];
    s = fma(cw, Xp[m * ldx + c], s);
    c += 256;
    while (c >= nocc) { c -= nocc; ++m; }
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) v[z * naux + P] = (red[0] + red[1]) + (red[2] + red[3]);
}

// J[z][i][j] = sum_P v[z][P] b^P_{ij}: one thread per packed pair, streaming B once.
constexpr int kCoulombZ = 4;
__global__ void __launch_bounds__(256) coulomb_kernel(const double* __restrict__ B, int64_t naux, int64_t nao,
                                                      int64_t npair, const double* __restrict__ v, int nz,
                                                      int64_t vstride, double* __restrict__ J, int64_t jstride) {
  __shared__ double vs[kCoulombZ][256];
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double acc[kCoulombZ] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t P0 = 0; P0 < naux; P0 += 256) {
    const int64_t cnt = naux - P0 < 256 ? naux - P0 : 256;
    __syncthreads();
    for (int z = 0; z < nz; ++z) vs[z][threadIdx.x] = threadIdx.x < cnt ? v[z * vstride + P0 + threadIdx.x] : 0.0;
    __syncthreads();
    if (p < npair) {
      const double* Bc = B + P0 * npair + p;
#pragma unroll 8
      for (int q = 0; q < cnt; ++q) {
        const double b = Bc[(int64_t)q * npair];
#pragma unroll
        for (int z = 0; z < kCoulombZ; ++z)
          if (z < nz) acc[z] = fma(vs[z][q], b, acc[z]);
      }
    }
  }
  if (p >= npair) return;
  int64_t i = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > p) --i;
  while ((i + 1) * (i + 2) / 2 <= p) ++i;
  const int64_t j = p - i * (i + 1) / 2;
  for (int z = 0; z < nz; ++z) {
    J[z * jstride + i * nao + j] = acc[z];
    J[z * jstride + j * nao + i] = acc[z];
  }
}

__global__ void __launch_bounds__(256) fill_zero_kernel(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------------------
// Launchers

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

hipError_t launch_half_transform(const double* B, int64_t naux, int64_t nao, const double* C,
                                 int64_t ldc, int64_t ncol, double* X, int64_t ldx, hipStream_t s) {
  typedef CfgBig Cg;
  // B operand: element (n = column of C, k = AO index) at C + k*ldc + n
  OpMap cm{C, ncol, ncol > 0 ? ncol : 1, 0, 1, 1, nao, 0, ldc, 0, nullptr, 0};
  const int64_t tm = cdiv(nao, Cg::BM), tn = cdiv(ncol, Cg::BN);
  const int64_t nblk = tm * tn * naux;
  if (nblk == 0) return hipSuccess;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  half_kernel<Cg><<<dim3((unsigned)nblk), dim3(Cg::NT), 0, s>>>(B, naux, (int)nao, nao * (nao + 1) / 2, cm,
                                                                 X, ldx, tm, tn);
  return hipGetLastError();
}

hipError_t launch_gemm(const OpMap& A, const OpMap& Bm, const OutMap& O, int64_t nz, hipStream_t s) {
  typedef CfgBig Cg;
  const int64_t tm = cdiv(O.M, Cg::BM), tn = cdiv(O.N, Cg::BN);
  if (tm * tn == 0 || nz == 0) return hipSuccess;
  if (tm * tn > 0x7fffffffLL || nz > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(tm * tn), 1, (unsigned)nz);
  const bool ak = A.s_kc == 1, bk = Bm.s_kc == 1;
  if (ak && bk) gemm_kernel<Cg, true, true><<<grid, Cg::NT, 0, s>>>(A, Bm, O, tm, tn);
  else if (ak) gemm_kernel<Cg, true, false><<<grid, Cg::NT, 0, s>>>(A, Bm, O, tm, tn);
  else if (bk) gemm_kernel<Cg, false, true><<<grid, Cg::NT, 0, s>>>(A, Bm, O, tm, tn);
  else gemm_kernel<Cg, false, false><<<grid, Cg::NT, 0, s>>>(A, Bm, O, tm, tn);
  return hipGetLastError();
}

int syrk_tile() { return CfgBig::BM; }

int syrk_splits(int64_t n, int64_t kb_n, int64_t nz) {
  const int64_t T = cdiv(n, CfgBig::BM);
  const int64_t work = T * (T + 1) / 2 * (nz > 0 ? nz : 1);
  int64_t ns = cdiv(1024, work);
  if (ns > kb_n) ns = kb_n;
  if (ns < 1) ns = 1;
  return (int)ns;
}

hipError_t launch_syrk_partial(const OpMap& A, const OpMap& Bw, int64_t n, int64_t nz, int nsplit,
                               double* Kpart, hipStream_t s) {
  typedef CfgBig Cg;
  const int64_t T = cdiv(n, Cg::BM);
  const int64_t npairs = T * (T + 1) / 2;
  if (npairs == 0 || nz == 0) return hipSuccess;
  if (nz > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(npairs * nsplit), 1, (unsigned)nz);
  syrk_kernel<Cg><<<grid, Cg::NT, 0, s>>>(A, Bw, n, nz, nsplit, npairs, Kpart);
  return hipGetLastError();
}

hipError_t launch_syrk_reduce(const double* Kpart, int nsplit, int64_t n, int64_t nz, double* K,
                              hipStream_t s) {
  const int64_t tot = n * n * nz;
  if (tot == 0) return hipSuccess;
  syrk_reduce_kernel<<<(unsigned)cdiv(tot, 256), 256, 0, s>>>(Kpart, nsplit, n, nz, K);
  return hipGetLastError();
}

hipError_t launch_jvec(const double* X, int64_t naux, int64_t nao, int64_t ldx, const double* C,
                       const double* w, int64_t nocc, int64_t nz, double* v, hipStream_t s) {
  if (naux == 0 || nz == 0) return hipSuccess;
  if (nz > 65535 || naux > 0x7fffffffLL) return hipErrorInvalidValue;
  jvec_kernel<<<dim3((unsigned)naux, (unsigned)nz), 256, 0, s>>>(X, nao, ldx, C, w, nocc, v, naux);
  return hipGetLastError();
}

hipError_t launch_coulomb(const double* B, int64_t naux, int64_t nao, const double* v, int64_t nz,
                          double* J, hipStream_t s) {
  const int64_t npair = nao * (nao + 1) / 2;
  for (int64_t z0 = 0; z0 < nz; z0 += kCoulombZ) {
    const int nzc = (int)(nz - z0 < kCoulombZ ? nz - z0 : kCoulombZ);
    coulomb_kernel<<<(unsigned)cdiv(npair, 256), 256, 0, s>>>(B, naux, nao, npair, v + z0 * naux, nzc, naux,
                                                               J + z0 * nao * nao, nao * nao);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_zero_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(p, n);
  return hipGetLastError();
}

}  // namespace dfk
