// HIP kernels for gfx950 (MI355X): FP64 contractions of the packed Cholesky tensor.
//
// Every dense contraction runs on the FP64 matrix cores (v_mfma_f64_16x16x4_f64,
// 64 cycles per issue per SIMD; one wave per SIMD can keep the unit busy).  Operand
// tiles go global -> registers -> LDS in a [row][k] layout with a row stride of 17
// doubles: the "k fastest" and "row fastest" global-load mappings both write, and the
// MFMA operand reads read, 32 lanes per LDS cycle without bank conflicts.
//
// Main loop: two LDS stages; the global loads of slab s+1 are issued before the MFMAs
// of slab s and written to the other stage after them, one barrier per slab.  Loads
// are branch-free (out-of-range elements read a valid address and are replaced by 0
// with a select), so no wait on outstanding loads sits between the prefetch and the
// MFMA block.
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
  static constexpr int LDS_A = BM * LD, LDS_B = BN * LD, STAGE = LDS_A + LDS_B;
  static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "tile must split evenly over threads");
};

// generic products and the K SYRK: 128 x 128 tiles, 2 x 2 waves of 64 x 64
typedef Cfg<2, 2, 4, 4> CfgSq;
// half transform: 128 rows x {176, 96, 48} columns, 4 waves stacked along the rows
typedef Cfg<4, 1, 2, 11> CfgH176;
typedef Cfg<4, 1, 2, 6> CfgH96;
typedef Cfg<4, 1, 2, 3> CfgH48;

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

// Two-stage software pipeline over nslab k-slabs.  load(s) fetches slab s into registers,
// store(stage) writes those registers into LDS stage `stage`.
template <class C, class FLoad, class FStore>
__device__ __forceinline__ void pipeline(double* smem, int64_t nslab, d4 (&acc)[C::TM][C::TN], int wm, int wn,
                                         int lane, FLoad&& load, FStore&& store) {
  if (nslab > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int64_t s = 0; s < nslab; ++s) {
    const int cur = (int)(s & 1);
    const bool more = s + 1 < nslab;
    if (more) load(s + 1);
    // keep the prefetch ahead of, and its consumers behind, the MFMA block
    __builtin_amdgcn_sched_barrier(0);
    mma_slab<C>(smem + cur * C::STAGE, smem + cur * C::STAGE + C::LDS_A, acc, wm, wn, lane);
    __builtin_amdgcn_sched_barrier(0);
    if (more) store(cur ^ 1);
    __syncthreads();
  }
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
    const uint32_t nh = o.s_nh ? (uint32_t)n / (uint32_t)o.nl : 0u;
    const int64_t noff = (int64_t)nh * o.s_nh + (n - (int64_t)nh * o.nl) * o.s_nl;
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + (wm * C::TM + i) * 16 + 4 * r + lg;
        const uint32_t mh = o.s_mh ? (uint32_t)m / (uint32_t)o.ml : 0u;
        if (m < o.M) base[(int64_t)mh * o.s_mh + (m - (int64_t)mh * o.ml) * o.s_ml + noff] = acc[i][j][r];
      }
  }
}

// Global -> register -> LDS loader for one operand described by an OpMap.
//   KC = true : lanes run along k (16 consecutive k of one row per 16 lanes)
//   KC = false: lanes run along the row index
//   SCALE     : multiply element (r, kc) by ks[z*s_ksz + kc] (applied when storing to LDS)
// The slab sequence is walked in order: kb outer, kc in chunks of 16 inner.
template <class C, int R, bool KC, bool SCALE = false>
struct Loader {
  static constexpr int E = R * C::BK / C::NT;
  static_assert(E <= 32, "validity mask holds 32 elements");
  int64_t rowbase[E];  // offset of (row, kb = 0, kc = 0), rows past the end clamped to the last one
  unsigned rowok;      // bit q: the row of element q exists
  double v[E];         // raw loaded values; invalid ones are zeroed when written to LDS
  double sc[SCALE ? E : 1];
  int64_t kso;
  int64_t kb;          // slab the next load() fetches: (kb, kc0)
  int kc0;
  int kvalid;          // valid k entries of the slab last loaded

  __device__ __forceinline__ static int rr(int t, int q) {
    const int e = t + C::NT * q;
    return KC ? e / C::BK : e % R;
  }
  __device__ __forceinline__ static int kk(int t, int q) {
    const int e = t + C::NT * q;
    return KC ? e % C::BK : e / R;
  }
  __device__ __forceinline__ void init(const OpMap& o, int64_t r0, int64_t z, int64_t kb0, int t) {
    kso = z * o.s_ksz;
    kb = kb0;
    kc0 = 0;
    kvalid = 0;
    rowok = 0;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int64_t r = r0 + rr(t, q);
      const bool ok = r < o.rows;
      rowok |= (ok ? 1u : 0u) << q;
      const uint32_t rc = (uint32_t)(ok ? r : o.rows - 1);   // row indices fit 32 bits
      uint32_t rh = 0, rlo = rc;
      if (o.s_rh != 0) {
        rh = rc / (uint32_t)o.rl;
        rlo = rc - rh * (uint32_t)o.rl;
      }
      rowbase[q] = z * o.s_z + (int64_t)rh * o.s_rh + (int64_t)rlo * o.s_rlo;
    }
  }
  // issue the loads of the current slab (addresses clamped in range) and advance
  __device__ __forceinline__ void load(const OpMap& o, int t) {
    const double* __restrict__ base = o.p + kb * o.s_kb;
    const int klast = (int)o.kc_n - 1;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int kc = min(kc0 + kk(t, q), klast);
      const int64_t koff = KC ? (int64_t)kc : (int64_t)(uint32_t)kc * (uint32_t)o.s_kc;
      v[q] = base[rowbase[q] + koff];
      if (SCALE) sc[q] = o.ks[kso + kc];
    }
    kvalid = (int)o.kc_n - kc0;
    kc0 += C::BK;
    if (kc0 >= o.kc_n) {
      kc0 = 0;
      ++kb;
    }
  }
  __device__ __forceinline__ void store(double* S, int t) const {
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const bool ok = ((rowok >> q) & 1u) && kk(t, q) < kvalid;
      const double x = SCALE ? v[q] * sc[q] : v[q];
      S[rr(t, q) * C::LD + kk(t, q)] = ok ? x : 0.0;
    }
  }
};

// ---------------------------------------------------------------------------------------
// Generic tiled product  C(m, n) = sum_k A(m, k) B(n, k)  over a batch (grid z).
template <class C, bool AK, bool BK>
__global__ void __launch_bounds__(C::NT) gemm_kernel(OpMap A, OpMap B, OutMap O, int64_t tilesM,
                                                     int64_t tilesN) {
  __shared__ double smem[2 * C::STAGE];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave % C::WM, wn = wave / C::WM;
  const int64_t tile = xcd_remap(blockIdx.x, tilesM * tilesN);
  const int64_t z = blockIdx.z;
  const int64_t m0 = (tile % tilesM) * C::BM, n0 = (tile / tilesM) * C::BN;

  Loader<C, C::BM, AK> la;
  Loader<C, C::BN, BK> lb;
  la.init(A, m0, z, 0, t);
  lb.init(B, n0, z, 0, t);
  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  const int64_t nslab = A.kb_n * ((A.kc_n + C::BK - 1) / C::BK);
  pipeline<C>(
      smem, nslab, acc, wm, wn, lane,
      [&](int64_t) {
        la.load(A, t);
        lb.load(B, t);
      },
      [&](int st) {
        la.store(smem + st * C::STAGE, t);
        lb.store(smem + st * C::STAGE + C::LDS_A, t);
      });
  store_tile<C>(O, z, m0, n0, acc, wm, wn, lane);
}

// ---------------------------------------------------------------------------------------
// Lower-triangle tile SYRK with the kb range split over workgroups:
// Kpart[split][z] tile (I, J), I >= J, = sum_{kb in split} sum_kc A(i, kb, kc) Bw(j, kb, kc),
// where Bw is A times an optional per-kc weight.
template <class C, bool SCALE>
__global__ void __launch_bounds__(C::NT) syrk_kernel(OpMap A, OpMap Bw, int64_t n, int64_t nz, int nsplit,
                                                     int64_t npairs, double* Kpart) {
  static_assert(C::BM == C::BN, "square tiles");
  __shared__ double smem[2 * C::STAGE];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave % C::WM, wn = wave / C::WM;
  const int64_t item = xcd_remap(blockIdx.x, npairs * nsplit);
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
  Loader<C, C::BN, true, SCALE> lb;
  la.init(A, m0, z, kb_lo, t);
  lb.init(Bw, n0, z, kb_lo, t);
  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  const int64_t nslab = (kb_hi - kb_lo) * ((A.kc_n + C::BK - 1) / C::BK);
  pipeline<C>(
      smem, nslab, acc, wm, wn, lane,
      [&](int64_t) {
        la.load(A, t);
        lb.load(Bw, t);
      },
      [&](int st) {
        la.store(smem + st * C::STAGE, t);
        lb.store(smem + st * C::STAGE + C::LDS_A, t);
      });
  OutMap o = out_plain(Kpart + ((int64_t)split * nz + z) * n * n, n, n, n);
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
// A operand element (m, k) = b^P_{mk}.  A slab strictly below the diagonal (every k < every
// m) is read along k: 16-element runs of packed rows.  Any other slab is read along m and
// addressed through (max, min), which for slabs above the diagonal are runs of packed row k.
// Packed offsets stay in 32 bits (nao <= 46340).
template <class C>
__global__ void __launch_bounds__(C::NT) half_kernel(const double* __restrict__ B, int64_t naux, int nao,
                                                     int64_t npair, OpMap Cm, double* __restrict__ X,
                                                     int64_t ldx, int64_t tilesM, int64_t tilesN) {
  __shared__ double smem[2 * C::STAGE];
  constexpr int EA = C::BM * C::BK / C::NT;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave % C::WM, wn = wave / C::WM;
  const int64_t ntile = tilesM * tilesN;
  const int64_t item = xcd_remap(blockIdx.x, ntile * naux);
  const int64_t P = item / ntile, tile = item % ntile;
  const int m0 = (int)((tile % tilesM) * C::BM), n0 = (int)((tile / tilesM) * C::BN);
  const double* __restrict__ Bp = B + P * npair;

  Loader<C, C::BN, false> lb;
  lb.init(Cm, n0, 0, 0, t);
  static_assert(EA <= 32, "validity mask holds 32 elements");
  static_assert(C::NT % C::BK == 0 && C::NT % C::BM == 0, "per-thread row / column of the A loads");
  // below-diagonal mapping: element q is row m0 + t/16 + q*NT/16, column k0 + t%16
  // other mapping:          element q is row m0 + t%BM,        column k0 + t/BM + q*NT/BM
  const unsigned last = (unsigned)nao - 1u;
  unsigned rowoffB[EA], rowokB = 0;
#pragma unroll
  for (int q = 0; q < EA; ++q) {
    const unsigned m = (unsigned)(m0 + (t + C::NT * q) / C::BK);
    rowokB |= (m <= last ? 1u : 0u) << q;
    const unsigned mc = m <= last ? m : last;
    rowoffB[q] = mc * (mc + 1u) / 2u + (unsigned)(t % C::BK);
  }
  const unsigned mA = (unsigned)(m0 + t % C::BM);
  const unsigned mAc = mA <= last ? mA : last;
  const unsigned mAoff = mAc * (mAc + 1u) / 2u;
  double va[EA];
  unsigned amask = 0;
  bool below = false;

  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  const int nslab = (nao + C::BK - 1) / C::BK;
  pipeline<C>(
      smem, nslab, acc, wm, wn, lane,
      [&](int64_t s) {
        const unsigned k0 = (unsigned)s * C::BK;
        below = (int)k0 + C::BK - 1 <= m0;
        if (below) {
          amask = rowokB;
#pragma unroll
          for (int q = 0; q < EA; ++q) va[q] = Bp[rowoffB[q] + k0];
        } else {
          amask = 0;
#pragma unroll
          for (int q = 0; q < EA; ++q) {
            const unsigned k = k0 + (unsigned)((t + C::NT * q) / C::BM);
            amask |= (mA <= last && k <= last ? 1u : 0u) << q;
            const unsigned kc = k <= last ? k : last;
            const unsigned idx = mAc >= kc ? mAoff + kc : kc * (kc + 1u) / 2u + mAc;
            va[q] = Bp[idx];
          }
        }
        lb.load(Cm, t);
      },
      [&](int st) {
        double* As = smem + st * C::STAGE;
#pragma unroll
        for (int q = 0; q < EA; ++q) {
          const int e = t + C::NT * q;
          const int slot = below ? (e / C::BK) * C::LD + e % C::BK : (e % C::BM) * C::LD + e / C::BM;
          As[slot] = ((amask >> q) & 1u) ? va[q] : 0.0;
        }
        lb.store(smem + st * C::STAGE + C::LDS_A, t);
      });
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
    while (c >= nocc) {
      c -= nocc;
      ++m;
    }
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

template <class Cg>
static hipError_t half_launch(const double* B, int64_t naux, int64_t nao, const OpMap& cm, double* X, int64_t ldx,
                              hipStream_t s) {
  const int64_t tm = cdiv(nao, Cg::BM), tn = cdiv(cm.rows, Cg::BN);
  const int64_t nblk = tm * tn * naux;
  if (nblk == 0) return hipSuccess;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  half_kernel<Cg><<<dim3((unsigned)nblk), dim3(Cg::NT), 0, s>>>(B, naux, (int)nao, nao * (nao + 1) / 2, cm, X, ldx,
                                                                 tm, tn);
  return hipGetLastError();
}

// Column tile of the half transform: the widest of {176, 96, 48} that pads ncol least.
int half_tile_n(int64_t ncol) {
  const int cands[3] = {176, 96, 48};
  int best = cands[0];
  int64_t best_pad = cdiv(ncol, best) * best;
  for (int c : cands) {
    const int64_t pad = cdiv(ncol, c) * c;
    if (pad < best_pad) {
      best = c;
      best_pad = pad;
    }
  }
  return best;
}

hipError_t launch_half_transform(const double* B, int64_t naux, int64_t nao, const double* C, int64_t ldc,
                                 int64_t ncol, double* X, int64_t ldx, hipStream_t s) {
  // B operand: element (n = column of C, k = AO index) at C + k*ldc + n
  const OpMap cm{C, ncol, ncol > 0 ? ncol : 1, 0, 1, 1, nao, 0, ldc, 0, nullptr, 0};
  switch (half_tile_n(ncol)) {
    case 176: return half_launch<CfgH176>(B, naux, nao, cm, X, ldx, s);
    case 96: return half_launch<CfgH96>(B, naux, nao, cm, X, ldx, s);
    default: return half_launch<CfgH48>(B, naux, nao, cm, X, ldx, s);
  }
}

hipError_t launch_gemm(const OpMap& A, const OpMap& Bm, const OutMap& O, int64_t nz, hipStream_t s) {
  typedef CfgSq Cg;
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

int syrk_tile() { return CfgSq::BM; }

int syrk_splits(int64_t n, int64_t kb_n, int64_t nz) {
  const int64_t T = cdiv(n, CfgSq::BM);
  const int64_t work = T * (T + 1) / 2 * (nz > 0 ? nz : 1);
  int64_t ns = cdiv(1024, work);
  if (ns > kb_n) ns = kb_n;
  if (ns < 1) ns = 1;
  return (int)ns;
}

hipError_t launch_syrk_partial(const OpMap& A, const OpMap& Bw, int64_t n, int64_t nz, int nsplit, double* Kpart,
                               hipStream_t s) {
  typedef CfgSq Cg;
  const int64_t T = cdiv(n, Cg::BM);
  const int64_t npairs = T * (T + 1) / 2;
  if (npairs == 0 || nz == 0) return hipSuccess;
  if (nz > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(npairs * nsplit), 1, (unsigned)nz);
  if (Bw.ks) syrk_kernel<Cg, true><<<grid, Cg::NT, 0, s>>>(A, Bw, n, nz, nsplit, npairs, Kpart);
  else syrk_kernel<Cg, false><<<grid, Cg::NT, 0, s>>>(A, Bw, n, nz, nsplit, npairs, Kpart);
  return hipGetLastError();
}

hipError_t launch_syrk_reduce(const double* Kpart, int nsplit, int64_t n, int64_t nz, double* K, hipStream_t s) {
  const int64_t tot = n * n * nz;
  if (tot == 0) return hipSuccess;
  syrk_reduce_kernel<<<(unsigned)cdiv(tot, 256), 256, 0, s>>>(Kpart, nsplit, n, nz, K);
  return hipGetLastError();
}

hipError_t launch_jvec(const double* X, int64_t naux, int64_t nao, int64_t ldx, const double* C, const double* w,
                       int64_t nocc, int64_t nz, double* v, hipStream_t s) {
  if (naux == 0 || nz == 0) return hipSuccess;
  if (nz > 65535 || naux > 0x7fffffffLL) return hipErrorInvalidValue;
  jvec_kernel<<<dim3((unsigned)naux, (unsigned)nz), 256, 0, s>>>(X, nao, ldx, C, w, nocc, v, naux);
  return hipGetLastError();
}

hipError_t launch_coulomb(const double* B, int64_t naux, int64_t nao, const double* v, int64_t nz, double* J,
                          hipStream_t s) {
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
