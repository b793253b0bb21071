// HIP kernels for gfx950 (MI355X): FP64 contractions of the packed Cholesky tensor.
//
// Every dense contraction runs on the FP64 matrix cores (v_mfma_f64_16x16x4_f64,
// 64 cycles per issue per SIMD; one wave per SIMD can keep the unit busy).  Operand
// tiles go global -> registers -> LDS in a [row][k] layout with a row stride of 17
// doubles.  The LDS serves 32 lanes of 8-byte accesses per cycle over 64 banks.  With this
// stride the "row fastest" stores are conflict-free; the "k fastest" stores and the MFMA
// operand reads have one colliding pair per 32 lanes.  An 18-double stride makes the reads
// conflict-free and the stores worse; the kernels run equally fast with either, because
// the conflicts hide behind the MFMAs.
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

#include <type_traits>
#include <utility>

namespace dfk {

typedef double d4 __attribute__((ext_vector_type(4)));

// WM x WN waves, each TM x TN MFMA tiles of 16 x 16; IL selects the interleaved schedule
// (loads and LDS stores spread between the MFMAs) over the bulk one.
template <int WM_, int WN_, int TM_, int TN_, bool IL_ = false>
struct Cfg {
  static constexpr int WM = WM_, WN = WN_, TM = TM_, TN = TN_;
  static constexpr bool IL = IL_;
  static constexpr int NT = 64 * WM * WN;
  static constexpr int BM = 16 * TM * WM, BN = 16 * TN * WN, BK = 16;
  static constexpr int LD = BK + 1;
  static constexpr int LDS_A = BM * LD, LDS_B = BN * LD, STAGE = LDS_A + LDS_B;
  static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "tile must split evenly over threads");
};

// Every MFMA kernel is sized for two waves per SIMD (at most 256 registers per lane, two
// workgroups' LDS per CU), so one wave's barrier and LDS latency hide behind the other's MFMAs.
// generic products and the K SYRK: 128 x 128 tiles, 2 x 2 waves of 64 x 64, interleaved
typedef Cfg<2, 2, 4, 4, true> CfgSq;
// tall products (M >= 256): 256 x 128 tiles, 4 x 2 waves of 64 x 64, one workgroup per CU; the
// same per-wave work with a quarter fewer loads per MFMA
typedef Cfg<4, 2, 4, 4, true> CfgTall;
typedef Cfg<2, 2, 4, 4, true> CfgSyrk;
// small matrices (fragment sizes): 64 x 64 SYRK tiles pad the triangle less
typedef Cfg<2, 2, 2, 2, true> CfgSyrk64;
// half transform: {64, 128, 128} rows x {176, 96, 48} columns, 4 waves stacked along the rows
typedef Cfg<4, 1, 1, 11, true> CfgH176;
typedef Cfg<4, 1, 2, 6> CfgH96;
typedef Cfg<4, 1, 2, 3> CfgH48;
// half transform on 2-D wave tiles: 128 rows x {128, 96, 64} columns, 2 x 2 waves of 4 x {4, 3, 2}
typedef Cfg<2, 2, 4, 4, true> CfgQ128;
typedef Cfg<2, 2, 4, 3, true> CfgQ96;
typedef Cfg<2, 2, 4, 2, true> CfgQ64;

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

// One k-step (4 deep) worth of MFMA operands of one wave.
template <class C>
struct Frag {
  double a[C::TM];
  double b[C::TN];
};

template <class C>
__device__ __forceinline__ void read_frag(const double* __restrict__ As, const double* __restrict__ Bs, int kk,
                                          Frag<C>& f, int wm, int wn, int lane) {
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int i = 0; i < C::TM; ++i) f.a[i] = As[((wm * C::TM + i) * 16 + lr) * C::LD + kk + lk];
#pragma unroll
  for (int j = 0; j < C::TN; ++j) f.b[j] = Bs[((wn * C::TN + j) * 16 + lr) * C::LD + kk + lk];
}

template <class C>
__device__ __forceinline__ void zero_acc(d4 (&acc)[C::TM][C::TN]) {
#pragma unroll
  for (int i = 0; i < C::TM; ++i)
#pragma unroll
    for (int j = 0; j < C::TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
}

// Compile-time loops.
template <int... I, class F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, I...>, F&& f) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

// Sources.  A source feeds both operand tiles of a product slab by slab:
//   begin()          set up the next slab (uniform values only)
//   load<q>()        issue global load q (of NL) of the slab
//   finish()         advance to the following slab (clamped at the last one)
//   store<q>(A, B)   write loaded element q to the LDS tiles A, B
// Rows and columns past the end of a matrix are read at clamped (valid) addresses and never
// zeroed: they only reach output rows and columns that are not stored.  Only contraction
// indices past the end (a partial last slab) must contribute zero.

// One slab of the software pipeline (interleaved schedule).  LDS stage `cur` holds the slab being
// multiplied and F[0] already holds its first k-step of operands.  While its TM*TN*BK/4 MFMAs
// issue one by one, the wave reads the operands of the next k-step, issues the global loads of
// the next slab in the first half and writes those registers to the other LDS stage in the
// second half.  Then one barrier and the first operands of the next slab.  Every slot is
// generated at compile time, so the body is one basic block; scheduling fences keep the
// interleave.  (One body per kernel: alternative slab bodies in one loop overflow the 256
// registers a lane has at two waves per SIMD.)
template <class C, class Src>
__device__ __forceinline__ void slab_step(Src& src, double* smem, int cur, d4 (&acc)[C::TM][C::TN], Frag<C> (&F)[2],
                                          int wm, int wn, int lane) {
  const double* As = smem + cur * C::STAGE;
  const double* Bs = As + C::LDS_A;
  double* An = smem + (cur ^ 1) * C::STAGE;
  double* Bn = An + C::LDS_A;
  constexpr int KS = C::BK / 4;            // k-steps per slab
  constexpr int PK = C::TM * C::TN;        // MFMAs per k-step
  constexpr int NM = PK * KS;              // MFMAs per slab
  constexpr int HALF = NM / 2;
  constexpr int NL = Src::NL;
  static_assert(HALF > 0, "at least two MFMAs per slab");
  src.begin();
  static_for<NM>([&](auto IDXc) {
    constexpr int IDX = decltype(IDXc)::value;
    constexpr int ks = IDX / PK, ij = IDX % PK, i = ij / C::TN, j = ij % C::TN;
    if constexpr (ij == 0) {
      if constexpr (ks + 1 < KS) read_frag<C>(As, Bs, (ks + 1) * 4, F[(ks + 1) & 1], wm, wn, lane);
      __builtin_amdgcn_sched_barrier(0);
    }
    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(F[ks & 1].a[i], F[ks & 1].b[j], acc[i][j], 0, 0, 0);
    if constexpr (IDX < HALF) {
      constexpr int Q0 = IDX * NL / HALF, Q1 = (IDX + 1) * NL / HALF;
      static_for<Q1 - Q0>([&](auto R) { src.template load<Q0 + decltype(R)::value>(); });
    } else {
      constexpr int Q0 = (IDX - HALF) * NL / HALF, Q1 = (IDX - HALF + 1) * NL / HALF;
      static_for<Q1 - Q0>([&](auto R) { src.template store<Q0 + decltype(R)::value>(An, Bn); });
    }
    __builtin_amdgcn_sched_barrier(0);
  });
  src.finish();
  __syncthreads();
  read_frag<C>(An, Bn, 0, F[0], wm, wn, lane);
}

// Bulk schedule of one slab: all global loads of the next slab, then every MFMA of this one,
// then the LDS stores of the loaded registers into the other stage and one barrier.
template <class C, class Src>
__device__ __forceinline__ void slab_step_bulk(Src& src, double* smem, int cur, d4 (&acc)[C::TM][C::TN], int wm,
                                               int wn, int lane) {
  const double* As = smem + cur * C::STAGE;
  const double* Bs = As + C::LDS_A;
  double* An = smem + (cur ^ 1) * C::STAGE;
  src.begin();
  static_for<Src::NL>([&](auto Q) { src.template load<decltype(Q)::value>(); });
  src.finish();
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int kk = 0; kk < C::BK; kk += 4) {
    Frag<C> f;
    read_frag<C>(As, Bs, kk, f, wm, wn, lane);
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int j = 0; j < C::TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(f.a[i], f.b[j], acc[i][j], 0, 0, 0);
  }
  __builtin_amdgcn_sched_barrier(0);
  static_for<Src::NL>([&](auto Q) { src.template store<decltype(Q)::value>(An, An + C::LDS_A); });
  __syncthreads();
}

// Runs nslab slabs through the pipeline (nslab >= 1).  The loads issued during the last slab
// re-read it (the sources clamp) and land in the stage nobody reads any more.
template <class C, class Src>
__device__ __forceinline__ void mainloop(Src& src, double* smem, int64_t nslab, d4 (&acc)[C::TM][C::TN], int wm,
                                         int wn, int lane) {
  src.begin();
  static_for<Src::NL>([&](auto Q) { src.template load<decltype(Q)::value>(); });
  src.finish();
  static_for<Src::NL>([&](auto Q) { src.template store<decltype(Q)::value>(smem, smem + C::LDS_A); });
  __syncthreads();
  if constexpr (C::IL) {
    Frag<C> F[2];
    read_frag<C>(smem, smem + C::LDS_A, 0, F[0], wm, wn, lane);
    for (int64_t s = 0; s < nslab; ++s) slab_step<C>(src, smem, (int)(s & 1), acc, F, wm, wn, lane);
  } else {
    for (int64_t s = 0; s < nslab; ++s) slab_step_bulk<C>(src, smem, (int)(s & 1), acc, wm, wn, lane);
  }
}

// Epilogue.  GEN = false stores the accumulators as they are (o.alpha must be 1 and
// o.accumulate 0); GEN = true applies alpha and accumulate.  Arithmetic on the accumulators
// here moves them out of the matrix-core registers for the whole main loop (a copy per MFMA
// operand per slab), so only launches that need it instantiate GEN.
template <class C, bool GEN>
__device__ __forceinline__ void store_tile(const OutMap& o, int64_t z, int64_t m0, int64_t n0,
                                           const d4 (&acc)[C::TM][C::TN], int wm, int wn, int lane) {
  const int lr = lane & 15, lg = lane >> 4;
  const int64_t zo1 = z * o.s_z, zo2 = z * o.s2_z;
#pragma unroll
  for (int j = 0; j < C::TN; ++j) {
    const int64_t n = n0 + (wn * C::TN + j) * 16 + lr;
    const bool nok = n < o.N, first = n < o.nsplit;
    const uint32_t nh = o.s_nh ? (uint32_t)n / (uint32_t)o.nl : 0u;
    const int64_t noff1 = (int64_t)nh * o.s_nh + (n - (int64_t)nh * o.nl) * o.s_nl;
    // integer select: p2 is null when every column goes to p
    const uintptr_t col = first ? (uintptr_t)o.p + 8u * (uint64_t)(zo1 + noff1)
                                : (uintptr_t)o.p2 + 8u * (uint64_t)(zo2 + n - o.nsplit);
#pragma unroll
    for (int i = 0; i < C::TM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + (wm * C::TM + i) * 16 + 4 * r + lg;
        const uint32_t mh = o.s_mh ? (uint32_t)m / (uint32_t)o.ml : 0u;
        const int64_t moff = first ? (int64_t)mh * o.s_mh + (m - (int64_t)mh * o.ml) * o.s_ml : m * o.s2_m;
        double* const dst = (double*)col + moff;
        if constexpr (GEN) {
          const double val = o.alpha * acc[i][j][r];
          if (nok && m < o.M) *dst = o.accumulate ? *dst + val : val;
        } else {
          if (nok && m < o.M) *dst = acc[i][j][r];
        }
      }
  }
}

// Operand described by an OpMap, staged through registers.  Slabs are walked in order (kb outer,
// kc in chunks of 16 inner) from slab `s_begin` to `s_end - 1`; the cursor stops at the last one.
//   KC = true : lanes run along k (16 consecutive k of one row per 16 lanes)
//   KC = false: lanes run along the row index
//   SCALE     : element (r, kc) times ks[z*s_ksz + kc]
//   CLAMP     : kc_n need not be a multiple of 16: in a partial slab k is clamped to the last
//               entry and entries past kc_n are zeroed.  Without CLAMP, every slab is read whole,
//               so kc_n must be a multiple of 16 or the rows padded with zeros up to one.
//   FLAT      : (KC only; no SCALE) the contraction index is flat, k = kb * kc_n + kc, and slab s
//               holds k in [16 s, 16 s + 16), running across kb blocks (kc_n >= 16: at most one
//               block boundary per slab), so kc_n need not be a multiple of 16 and no slab is
//               padded but the last of the whole contraction; slab numbers s_begin, s_end count
//               these flat slabs.
// Element q of a thread sits at base + eoff[q] with base uniform per slab, so without CLAMP a
// slab costs no per-element arithmetic.
template <class C, int R, bool KC, bool SCALE = false, bool CLAMP = true, bool FLAT = false>
struct Operand {
  static_assert(!FLAT || (KC && !SCALE), "flat contraction: lanes along k, no weights");
  static constexpr int E = R * C::BK / C::NT;
  uint32_t eoff[E];     // offset of element q from the slab base (row clamped to the last one)
  double v[E];
  double sc[SCALE ? E : 1];
  int kval;             // valid k entries of the slab set up by begin() (FLAT: entries before the block boundary)
  const double* base;
  const double* cur;    // start of the next slab to load (kept up to date by finish: no multiplies per slab)
  const double* ksb;
  int64_t zoff, kso;
  int64_t kb, kb_last;  // cursor: next slab to load is (kb, kc0)
  int kc0, kc_last;
  int64_t krem;         // FLAT: entries of the contraction from the next slab's start to its end
  int rem;              // FLAT: valid entries of the slab set up by begin()
  uint32_t dwrap;       // FLAT: s_kb - kc_n s_kc, from entry (kb, kc_n + j) to (kb + 1, j)

  __device__ __forceinline__ static int rr(int t, int q) {
    const int e = t + C::NT * q;
    return KC ? e / C::BK : e % R;
  }
  __device__ __forceinline__ static int kk(int t, int q) {
    const int e = t + C::NT * q;
    return KC ? e % C::BK : e / R;
  }
  // rows [r0, r0 + R) of batch z
  __device__ __forceinline__ void init(const OpMap& o, int64_t r0, int64_t z, int64_t s_begin, int64_t s_end,
                                       int t) {
    zoff = z * o.s_z;
    kso = z * o.s_ksz;
    if constexpr (FLAT) {
      const int64_t k0 = s_begin * C::BK, kl = (s_end - 1) * C::BK;
      kb = k0 / o.kc_n;
      kc0 = (int)(k0 - kb * o.kc_n);
      kb_last = kl / o.kc_n;
      kc_last = (int)(kl - kb_last * o.kc_n);
      krem = o.kb_n * o.kc_n - k0;
      dwrap = (uint32_t)(o.s_kb - o.kc_n * o.s_kc);
    } else {
      const int64_t nkc = (o.kc_n + C::BK - 1) / C::BK;
      kb = s_begin / nkc;
      kc0 = (int)(s_begin % nkc) * C::BK;
      kb_last = (s_end - 1) / nkc;
      kc_last = (int)((s_end - 1) % nkc) * C::BK;
    }
    cur = o.p + zoff + kb * o.s_kb + (int64_t)kc0 * o.s_kc;
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int64_t r = r0 + rr(t, q);
      const uint32_t rc = (uint32_t)(r < o.rows ? r : o.rows - 1);
      uint32_t rh = 0, rlo = rc;
      if (o.s_rh != 0) {
        rh = rc / (uint32_t)o.rl;
        rlo = rc - rh * (uint32_t)o.rl;
      }
      eoff[q] = rh * (uint32_t)o.s_rh + rlo * (uint32_t)o.s_rlo + (uint32_t)kk(t, q) * (uint32_t)o.s_kc;
    }
  }
  __device__ __forceinline__ void begin(const OpMap& o) {
    base = cur;
    kval = (int)o.kc_n - kc0;
    if constexpr (FLAT) rem = krem < C::BK ? (int)krem : C::BK;
    if constexpr (SCALE) ksb = o.ks + kso + kc0;
  }
  template <int q>
  __device__ __forceinline__ void load(const OpMap& o, int t) {
    if constexpr (FLAT) {
      // entries past the block boundary continue in the next kb block; entries past the end of
      // the contraction read the slab's first entry (row 0, in bounds; zeroed in store)
      const int kq = kk(t, q);
      const uint32_t off = eoff[q] + (kq >= kval ? dwrap : 0u);
      v[q] = base[kq < rem ? off : 0u];
    } else if constexpr (!CLAMP) {
      v[q] = base[eoff[q]];
      if constexpr (SCALE) sc[q] = ksb[kk(t, q)];
    } else {
      // entries past kc_n read the last valid k of the row instead (zeroed in store)
      const int over = kk(t, q) - (kval - 1);
      const uint32_t back = over > 0 ? (uint32_t)over * (uint32_t)o.s_kc : 0u;
      v[q] = base[eoff[q] - back];
      if constexpr (SCALE) sc[q] = ksb[min(kk(t, q), kval - 1)];
    }
  }
  __device__ __forceinline__ void finish(const OpMap& o) {
    // advance the cursor, but never past the last slab
    const bool at_end = kb == kb_last && kc0 == kc_last;
    if constexpr (FLAT) {
      int nkc = kc0 + C::BK;
      int64_t nkb = kb, step = (int64_t)C::BK * o.s_kc;
      if (nkc >= o.kc_n) {
        nkc -= (int)o.kc_n;
        ++nkb;
        step += o.s_kb - o.kc_n * o.s_kc;
      }
      kc0 = at_end ? kc0 : nkc;
      kb = at_end ? kb : nkb;
      cur = at_end ? cur : cur + step;
      krem = at_end ? krem : krem - C::BK;
      return;
    }
    int nkc = kc0 + C::BK;
    int64_t nkb = kb;
    // the next slab starts BK columns on, or at column 0 of the next kb block
    int64_t step = (int64_t)C::BK * o.s_kc;
    if (nkc >= o.kc_n) {
      nkc = 0;
      ++nkb;
      step = o.s_kb - (int64_t)kc0 * o.s_kc;
    }
    kc0 = at_end ? kc0 : nkc;
    kb = at_end ? kb : nkb;
    cur = at_end ? cur : cur + step;
  }
  template <int q>
  __device__ __forceinline__ void store(double* Sm, int t) const {
    const double x = SCALE ? v[q] * sc[q] : v[q];
    const int slot = rr(t, q) * C::LD + kk(t, q);
    if constexpr (FLAT) Sm[slot] = kk(t, q) < rem ? x : 0.0;
    else if constexpr (!CLAMP) Sm[slot] = x;
    else Sm[slot] = kk(t, q) < kval ? x : 0.0;
  }
};

// Source of a product with both operands from OpMaps over the same slab sequence.
template <class C, bool AK, bool BK, bool SCALE, bool CLAMP, bool FLAT = false>
struct PairSrc {
  static constexpr int EA = Operand<C, C::BM, AK, false, CLAMP, FLAT>::E;
  static constexpr int NL = EA + Operand<C, C::BN, BK, SCALE, CLAMP, FLAT>::E;
  Operand<C, C::BM, AK, false, CLAMP, FLAT> a;
  Operand<C, C::BN, BK, SCALE, CLAMP, FLAT> b;
  const OpMap* A;
  const OpMap* B;
  int t;
  __device__ __forceinline__ void begin() {
    a.begin(*A);
    b.begin(*B);
  }
  template <int q>
  __device__ __forceinline__ void load() {
    if constexpr (q < EA) a.template load<q>(*A, t);
    else b.template load<q - EA>(*B, t);
  }
  __device__ __forceinline__ void finish() {
    a.finish(*A);
    b.finish(*B);
  }
  template <int q>
  __device__ __forceinline__ void store(double* As, double* Bs) const {
    if constexpr (q < EA) a.template store<q>(As, t);
    else b.template store<q - EA>(Bs, t);
  }
};

// ---------------------------------------------------------------------------------------
// Generic tiled product  C(m, n) = sum_k A(m, k) B(n, k)  over a batch (grid z).  With grid
// y = nsplit > 1 each workgroup set covers a contiguous range of k slabs and writes its partial
// sums to part[split][M][N] (nz must be 1 then).
// Output tile (m0, n0) of batch z, split `split` of nsplit (partials to part when given).
template <class C, bool AK, bool BK, bool GEN, bool CLAMP>
__device__ __forceinline__ void gemm_tile(const OpMap& A, const OpMap& B, const OutMap& O, int64_t m0, int64_t n0,
                                          int64_t z, int nsplit, int split, double* part, double* smem) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave % C::WM, wn = wave / C::WM;
  const int64_t nslab_all = A.kb_n * ((A.kc_n + C::BK - 1) / C::BK);
  const int64_t s0 = nslab_all * split / nsplit, s1 = nslab_all * (split + 1) / nsplit;

  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  if (s1 > s0) {
    PairSrc<C, AK, BK, false, CLAMP> src;
    src.A = &A;
    src.B = &B;
    src.t = t;
    src.a.init(A, m0, z, s0, s1, t);
    src.b.init(B, n0, z, s0, s1, t);
    mainloop<C>(src, smem, s1 - s0, acc, wm, wn, lane);
  }
  if (part) {
    const OutMap po = out_plain(part + (int64_t)split * O.M * O.N, O.M, O.N, O.N);
    store_tile<C, false>(po, 0, m0, n0, acc, wm, wn, lane);
  } else {
    store_tile<C, GEN>(O, z, m0, n0, acc, wm, wn, lane);
  }
}

template <class C, bool AK, bool BK, bool GEN, bool CLAMP>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2))) gemm_kernel(OpMap A, OpMap B, OutMap O, int64_t tilesM, int64_t tilesN,
                                                     double* part) {
  __shared__ double smem[2 * C::STAGE];
  const int64_t tile = xcd_remap(blockIdx.x, tilesM * tilesN);
  const int64_t m0 = (tile % tilesM) * C::BM, n0 = (tile / tilesM) * C::BN;
  gemm_tile<C, AK, BK, GEN, CLAMP>(A, B, O, m0, n0, blockIdx.z, gridDim.y, blockIdx.y, part, smem);
}

// Rows in whole 128-row bands on 128 x 128 tiles and the rest (at most 64 rows) on 64 x 128 tiles
// (4 waves of 64 x 32), in one launch: per column block the band tiles, then the tail tile.
// Where the 256 x 128 or 128 x 128 tiles would pad the rows by more than 64 (1200 rows: 1280).
typedef Cfg<1, 4, 4, 2, true> CfgRowTail;
template <bool AK, bool BK>
__global__ void __launch_bounds__(CfgSq::NT) __attribute__((amdgpu_waves_per_eu(2))) gemm_tail_kernel(OpMap A, OpMap B, OutMap O, int64_t nband, int64_t tilesN) {
  static_assert(CfgRowTail::NT == CfgSq::NT && CfgRowTail::BN == CfgSq::BN && CfgRowTail::STAGE <= CfgSq::STAGE,
                "one workgroup shape and column block");
  __shared__ double smem[2 * CfgSq::STAGE];
  const int64_t per = nband + 1;
  const int64_t tile = xcd_remap(blockIdx.x, per * tilesN);
  const int64_t i = tile % per, n0 = (tile / per) * CfgSq::BN;
  if (i < nband)
    gemm_tile<CfgSq, AK, BK, false, false>(A, B, O, i * CfgSq::BM, n0, 0, 1, 0, nullptr, smem);
  else
    gemm_tile<CfgRowTail, AK, BK, false, false>(A, B, O, nband * CfgSq::BM, n0, 0, 1, 0, nullptr, smem);
}

// C(m, n) = alpha * sum_s part[s][m][n] (+ C), fixed order over s.
__global__ void __launch_bounds__(256) split_reduce_kernel(const double* __restrict__ part, int nsplit, OutMap O) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t MN = O.M * O.N;
  if (idx >= MN) return;
  const int64_t m = idx / O.N, n = idx % O.N;
  double s = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) s += part[(int64_t)sp * MN + idx];
  double* dst;
  if (n < O.nsplit) {
    dst = O.p + (m / O.ml) * O.s_mh + (m % O.ml) * O.s_ml + (n / O.nl) * O.s_nh + (n % O.nl) * O.s_nl;
  } else {
    dst = O.p2 + m * O.s2_m + (n - O.nsplit);
  }
  *dst = O.accumulate ? *dst + O.alpha * s : O.alpha * s;
}

// ---------------------------------------------------------------------------------------
// Lower-triangle tile SYRK with the kb range split over workgroups:
// Kpart[split][z] tile (I, J), I >= J, = sum_{kb in split} sum_kc A(i, kb, kc) Bw(j, kb, kc),
// where Bw is A times an optional per-kc weight.
// One (tile pair, split) item of density z.  FLAT: the contraction (kb, kc) runs as one flat
// index in slabs of 16 (see Operand) and the flat slabs are split evenly, so no kb block is padded
// to whole slabs; otherwise the kb range is split and each block padded.
template <class C, bool SCALE, bool CLAMP, bool FLAT = false>
__device__ __forceinline__ void syrk_tile(const OpMap& A, const OpMap& Bw, int64_t n, int64_t nz, int nsplit,
                                          int64_t npairs, double* Kpart, int64_t item, int64_t z, double* smem) {
  static_assert(C::BM == C::BN, "square tiles");
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave % C::WM, wn = wave / C::WM;
  const int64_t pair = item % npairs;
  const int split = (int)(item / npairs);
  // triangular decode: pair = I(I+1)/2 + J, 0 <= J <= I
  int64_t I = (int64_t)((sqrt(8.0 * (double)pair + 1.0) - 1.0) * 0.5);
  while (I * (I + 1) / 2 > pair) --I;
  while ((I + 1) * (I + 2) / 2 <= pair) ++I;
  const int64_t J = pair - I * (I + 1) / 2;
  const int64_t m0 = I * C::BM, n0 = J * C::BN;
  int64_t s_lo, s_hi;   // slabs of this split
  if constexpr (FLAT) {
    const int64_t S = (A.kb_n * A.kc_n + C::BK - 1) / C::BK;
    s_lo = S * split / nsplit;
    s_hi = S * (split + 1) / nsplit;
  } else {
    const int64_t nkc = (A.kc_n + C::BK - 1) / C::BK;
    s_lo = A.kb_n * split / nsplit * nkc;
    s_hi = A.kb_n * (split + 1) / nsplit * nkc;
  }

  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  const int64_t nslab = s_hi - s_lo;
  if (nslab > 0) {
    PairSrc<C, true, true, SCALE, CLAMP, FLAT> src;
    src.A = &A;
    src.B = &Bw;
    src.t = t;
    src.a.init(A, m0, z, s_lo, s_hi, t);
    src.b.init(Bw, n0, z, s_lo, s_hi, t);
    mainloop<C>(src, smem, nslab, acc, wm, wn, lane);
  }
  OutMap o = out_plain(Kpart + ((int64_t)split * nz + z) * n * n, n, n, n);
  store_tile<C, false>(o, 0, m0, n0, acc, wm, wn, lane);
}

template <class C, bool SCALE, bool CLAMP, bool FLAT = false>
__global__ void __launch_bounds__(C::NT) syrk_kernel(OpMap A, OpMap Bw, int64_t n, int64_t nz, int nsplit,
                                                     int64_t npairs, double* Kpart) {
  __shared__ double smem[2 * C::STAGE];
  syrk_tile<C, SCALE, CLAMP, FLAT>(A, Bw, n, nz, nsplit, npairs, Kpart, xcd_remap(blockIdx.x, npairs * nsplit),
                                   blockIdx.z, smem);
}

// Grouped K SYRK: problem p owns items [start[p], start[p + 1]) = (density z, split, tile pair),
// z outermost; unit weights.
struct SyrkDesc {
  OpMap A;
  int64_t n, nz, npairs;
  double* Kpart;
  int nsplit;
};
struct SyrkGroup {
  int n;
  int64_t start[kMaxGroup + 1];
  int64_t xs[9];   // items of XCD x: [xs[x], xs[x + 1])
  SyrkDesc d[kMaxGroup];
};

// With the per-XCD chunks of half_group_kernel.
template <class C, bool CLAMP, bool FLAT = false>
__global__ void __launch_bounds__(C::NT) syrk_group_kernel(SyrkGroup g) {
  __shared__ double smem[2 * C::STAGE];
  const int x = blockIdx.x % 8;
  const int64_t it = g.xs[x] + blockIdx.x / 8;
  if (it >= g.xs[x + 1]) return;
  int p = 0;
  while (p + 1 < g.n && it >= g.start[p + 1]) ++p;
  const SyrkDesc& d = g.d[p];
  const int64_t item = it - g.start[p], per_z = d.npairs * d.nsplit;
  syrk_tile<C, false, CLAMP, FLAT>(d.A, d.A, d.n, d.nz, d.nsplit, d.npairs, d.Kpart, item % per_z, item / per_z,
                                   smem);
}

__global__ void __launch_bounds__(256) syrk_reduce_kernel(const double* __restrict__ Kpart, int nsplit,
                                                          int64_t n, int64_t nz, double* __restrict__ K,
                                                          int accumulate) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nn = n * n;
  if (idx >= nn * nz) return;
  const int64_t z = idx / nn, rem = idx % nn, i = rem / n, j = rem % n;
  const int64_t a = i >= j ? i : j, b = i >= j ? j : i;   // the lower element, computed by the SYRK tiles
  double s = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) s += Kpart[((int64_t)sp * nz + z) * nn + a * n + b];
  K[idx] = accumulate ? K[idx] + s : s;
}

// ---------------------------------------------------------------------------------------
// Half transform of one packed, symmetric b^P against a dense C.
// A operand element (m, k) = b^P_{mk}, packed at T(max(m, k)) + min(m, k), T(i) = i(i+1)/2.
// A slab wholly below the diagonal of its row band (k0 + 15 <= m0: every k <= every m) is read
// along k, as 16-element runs of packed rows m: T(m) + k0 + (t % 16), a uniform base plus a
// per-thread constant.  Any other slab is read along m through (max, min); there k is uniform
// per wave and element, so T(k) is scalar work.  Both addresses are formed and a uniform select
// picks one.  The dense operand (C, or Y in the P-summed form) is read without clamping: its k
// extent must be padded with zero rows to a multiple of 16, which also cancels the clamped
// duplicates of b^P read for k past the end.  Packed offsets stay in 32 bits (nao <= 46340).
template <class C>
struct HalfSrc {
  static constexpr int EA = C::BM * C::BK / C::NT;
  static constexpr int NL = EA + Operand<C, C::BN, false, false, false>::E;
  static_assert(C::NT % C::BK == 0 && C::NT % C::BM == 0, "per-thread row / column of the A loads");
  static_assert(C::BM % 64 == 0, "t / BM is the same for all lanes of a wave");
  Operand<C, C::BN, false, false, false> c;
  const OpMap* Cm;
  const double* Bbase;  // packed b^P of the current P: Bbase + P*npair
  const double* Bp;
  int64_t npair, P, P_last;
  unsigned last;        // nao - 1
  int m0, t, nks, ks;   // k slabs per P, current k slab
  unsigned k0, kw;      // slab start; wave-uniform k offset t / BM of the along-m mapping
  bool below;
  uint32_t offB[EA];    // along-k mapping: T(m) + t % 16 for row m = m0 + e / 16 (clamped)
  uint32_t mAc, mAoff;  // along-m mapping: row m0 + t % BM (clamped) and T of it
  double va[EA];

  // slabs run over P in [P0, P1) (outer) and the k chunks of nao (inner)
  __device__ __forceinline__ void init(const double* B, int64_t npair_, int64_t P0, int64_t P1, int nao, int m0_,
                                       int t_) {
    Bbase = B;
    npair = npair_;
    P = P0;
    P_last = P1 - 1;
    last = (unsigned)nao - 1u;
    m0 = m0_;
    t = t_;
    nks = (nao + C::BK - 1) / C::BK;
    ks = 0;
    Bp = Bbase + P * npair;
#pragma unroll
    for (int q = 0; q < EA; ++q) {
      const unsigned m = (unsigned)(m0 + (t + C::NT * q) / C::BK);
      const unsigned mc = m <= last ? m : last;
      offB[q] = mc * (mc + 1u) / 2u + (unsigned)(t % C::BK);
    }
    const unsigned mA = (unsigned)(m0 + t % C::BM);
    mAc = mA <= last ? mA : last;
    mAoff = mAc * (mAc + 1u) / 2u;
    kw = (unsigned)__builtin_amdgcn_readfirstlane(t / C::BM);
  }
  __device__ __forceinline__ void begin() {
    k0 = (unsigned)ks * C::BK;
    below = (int)k0 + C::BK - 1 <= m0;
    c.begin(*Cm);
  }
  template <int q>
  __device__ __forceinline__ void load() {
    if constexpr (q < EA) {
      const unsigned kr = k0 + kw + (unsigned)(q * (C::NT / C::BM));   // uniform
      const unsigned kc = kr <= last ? kr : last;
      const unsigned Tk = kc * (kc + 1u) / 2u;
      // bit-mask blends: conditionals here compile to a divergent branch (per lane) or to uniform
      // branches (on `below`) per load
      const unsigned sel = 0u - (unsigned)(mAc >= kc);
      const unsigned other = ((mAoff + kc) & sel) | ((Tk + mAc) & ~sel);
      const unsigned bsel = 0u - (unsigned)below;
      va[q] = Bp[((offB[q] + k0) & bsel) | (other & ~bsel)];
    } else {
      c.template load<q - EA>(*Cm, t);
    }
  }
  __device__ __forceinline__ void finish() {
    const bool at_end = P == P_last && ks == nks - 1;
    int nk = ks + 1;
    int64_t nP = P;
    if (nk == nks) {
      nk = 0;
      ++nP;
    }
    ks = at_end ? ks : nk;
    Bp = at_end || nP == P ? Bp : Bp + npair;
    P = at_end ? P : nP;
    c.finish(*Cm);
  }
  template <int q>
  __device__ __forceinline__ void store(double* As, double* Bs) const {
    if constexpr (q < EA) {
      const int e = t + C::NT * q;
      As[below ? (e / C::BK) * C::LD + e % C::BK : (e % C::BM) * C::LD + e / C::BM] = va[q];
    } else {
      c.template store<q - EA>(Bs, t);
    }
  }
};

// The J-vector of Eq. (J_1) formed in the half transform's epilogue: with X_P = b^P C the tile
// just computed, v_P = sum_{m < nao, c < nv} X_P[m][c] C[m][c] w[c] (w NULL: all ones), since
// sum_c X_P[m][c] C[m][c] w[c] summed over m is <b^P, C diag(w) C^T>.  Each tile leaves its
// partial sum in part[P * tiles + tile]; jv_reduce_kernel adds them up in tile order.
struct JvEpi {
  const double* C;   // C[m * ldc + c], the operand of the half transform (L2-resident: the main loop read it)
  int64_t ldc;
  const double* w;
  int nv;
  double* part;      // partial of tile `tile` of P at part[P * T + toff + tile]
  int64_t T, toff;
};

// The output tile of b^P at (m0, n0); with JV its J-vector partial goes to slot `tile` of P.
template <class C, bool GEN = false, bool JV = false>
__device__ __forceinline__ void half_tile_at(const double* __restrict__ B, int nao, int64_t npair, const OpMap& Cm,
                                             const OutMap& out, int64_t P, int m0, int n0, int64_t tile,
                                             double* smem, const JvEpi* jv) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave % C::WM, wn = wave / C::WM;
  const int nslab = (nao + C::BK - 1) / C::BK;

  HalfSrc<C> src;
  src.Cm = &Cm;
  src.c.init(Cm, n0, 0, 0, nslab, t);
  src.init(B, npair, P, P + 1, nao, m0, t);
  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  mainloop<C>(src, smem, nslab, acc, wm, wn, lane);
  store_tile<C, GEN>(out, P, m0, n0, acc, wm, wn, lane);
  if constexpr (JV) {
    const int lr = lane & 15, lg = lane >> 4;
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < C::TN; ++j) {
      const int n = n0 + (wn * C::TN + j) * 16 + lr;
      const bool nok = n < jv->nv;
      const int nc = nok ? n : 0;
      const double wc = nok ? (jv->w ? jv->w[nc] : 1.0) : 0.0;
      double sj = 0.0;
#pragma unroll
      for (int i = 0; i < C::TM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + (wm * C::TM + i) * 16 + 4 * r + lg;
          const double cm = m < nao ? jv->C[(int64_t)m * jv->ldc + nc] : 0.0;
          sj = fma(acc[i][j][r], cm, sj);
        }
      s = fma(sj, wc, s);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    __syncthreads();   // the main loop's last LDS reads are done before smem is reused
    if (lane == 0) smem[wave] = s;
    __syncthreads();
    if (t == 0) {
      double r = 0.0;
      for (int q = 0; q < C::WM * C::WN; ++q) r += smem[q];
      jv->part[P * jv->T + jv->toff + tile] = r;
    }
  }
}

// One output tile (item = P * tiles + tile) of the half transform; row bands start at row r0.
template <class C, bool GEN = false, bool JV = false>
__device__ __forceinline__ void half_tile(const double* __restrict__ B, int nao, int64_t npair, const OpMap& Cm,
                                          const OutMap& out, int64_t tilesM, int64_t tilesN, int64_t item, int r0,
                                          double* smem, const JvEpi* jv = nullptr) {
  const int64_t ntile = tilesM * tilesN;
  // row band major: the column tiles of one band of b^P run side by side and share its reads in L2
  const int64_t P = item / ntile, tile = item % ntile;
  const int m0 = r0 + (int)((tile / tilesN) * C::BM), n0 = (int)((tile % tilesN) * C::BN);
  half_tile_at<C, GEN, JV>(B, nao, npair, Cm, out, P, m0, n0, tile, smem, jv);
}

// Rows [r0, r0 + tilesM * 128) on two tile shapes in one launch: per row band, nA tiles of CA
// (columns [0, nA CA::BN)) and one of CB (the remainder columns from nA CA::BN on).  The tiles of
// one band of b^P run side by side and share its reads in L2, which two launches would not.
template <class CA, class CB, bool GEN, bool JV>
__global__ void __launch_bounds__(CA::NT) __attribute__((amdgpu_waves_per_eu(2))) half_pair_kernel(const double* __restrict__ B, int64_t naux, int nao,
                                                          int64_t npair, OpMap Cm, OutMap out, int64_t tilesM,
                                                          int64_t nA, int r0, JvEpi jv) {
  static_assert(CA::BM == CB::BM && CA::NT == CB::NT, "one row band, one workgroup shape");
  __shared__ double smem[2 * (CA::STAGE > CB::STAGE ? CA::STAGE : CB::STAGE)];
  const int64_t per = nA + 1, ntile = tilesM * per;
  const int64_t item = xcd_remap(blockIdx.x, ntile * naux);
  const int64_t P = item / ntile, tile = item % ntile, j = tile % per;
  const int m0 = r0 + (int)((tile / per) * CA::BM);
  if (j < nA)
    half_tile_at<CA, GEN, JV>(B, nao, npair, Cm, out, P, m0, (int)(j * CA::BN), tile, smem, &jv);
  else
    half_tile_at<CB, GEN, JV>(B, nao, npair, Cm, out, P, m0, (int)(nA * CA::BN), tile, smem, &jv);
}

// GEN: the epilogue applies out.alpha and out.accumulate (a separate instantiation, see store_tile)
template <class C, bool GEN>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2))) half_kernel(const double* __restrict__ B, int64_t naux, int nao,
                                                     int64_t npair, OpMap Cm, OutMap out, int64_t tilesM,
                                                     int64_t tilesN, int r0) {
  __shared__ double smem[2 * C::STAGE];
  half_tile<C, GEN>(B, nao, npair, Cm, out, tilesM, tilesN, xcd_remap(blockIdx.x, tilesM * tilesN * naux), r0, smem);
}

// The half transform with the J-vector partials in its epilogue (JvEpi).
template <class C>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2))) half_jv_kernel(const double* __restrict__ B, int64_t naux, int nao,
                                                        int64_t npair, OpMap Cm, OutMap out, int64_t tilesM,
                                                        int64_t tilesN, int r0, JvEpi jv) {
  __shared__ double smem[2 * C::STAGE];
  half_tile<C, false, true>(B, nao, npair, Cm, out, tilesM, tilesN, xcd_remap(blockIdx.x, tilesM * tilesN * naux),
                            r0, smem, &jv);
}

// v[P] (+)= sum_{t < tiles} part[P * tiles + t], in tile order.
__global__ void __launch_bounds__(256) jv_reduce_kernel(const double* __restrict__ part, int64_t tiles, int64_t naux,
                                                        double* __restrict__ v, int accumulate) {
  const int64_t P = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (P >= naux) return;
  const double* q = part + P * tiles;
  double s = 0.0;
  for (int64_t t = 0; t < tiles; ++t) s += q[t];
  v[P] = accumulate ? v[P] + s : s;
}

// Grouped half transform over several problems in one launch.  Work items of problem p are
// [start[p], start[p + 1]); problems are listed largest first, so the big ones start first and
// the small ones fill in behind them.
struct HalfDesc {
  const double* B;
  int64_t npair, tilesM, tilesN;
  OpMap Cm;
  OutMap out;
  int nao, r0;   // row bands from row r0
};
struct HalfGroup {
  int n;
  int64_t start[kMaxGroup + 1];
  int64_t xs[9];   // items of XCD x: [xs[x], xs[x + 1])
  HalfDesc d[kMaxGroup];
};

// Grouped launches: the item list is cut into 8 contiguous chunks of about equal cost, one per
// XCD.  The dispatcher deals workgroups to the 8 XCDs in turn, so workgroup b runs on XCD b % 8
// and takes item b / 8 of that XCD's chunk (workgroups past the end of their chunk exit):
// consecutive items run side by side on one XCD and share its L2, and every XCD gets the same
// work although the items of different problems differ in cost.  (A persistent grid striding
// through the chunks balanced uneven items worse than the dispatcher does.)
template <class C>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2))) half_group_kernel(HalfGroup g) {
  __shared__ double smem[2 * C::STAGE];
  const int x = blockIdx.x % 8;
  const int64_t item = g.xs[x] + blockIdx.x / 8;
  if (item >= g.xs[x + 1]) return;
  int p = 0;
  while (p + 1 < g.n && item >= g.start[p + 1]) ++p;
  const HalfDesc& d = g.d[p];
  half_tile<C>(d.B, d.nao, d.npair, d.Cm, d.out, d.tilesM, d.tilesN, item - g.start[p], d.r0, smem);
}

// part[split] (m, n) = sum_{P in split} sum_k b^P_{mk} Y(n, (P, k)): the packed half-transform
// product with the right operand changing with P and the P sum split over grid y.
// Row bands start at row r0; part[split] holds rows [r0, r0 + tilesM * BM) clipped to nao, as
// [nao - r0 clipped][N] with N = Y.rows.
template <class C>
__global__ void __launch_bounds__(C::NT) __attribute__((amdgpu_waves_per_eu(2))) half_reduce_kernel(const double* __restrict__ B, int64_t naux, int nao,
                                                            int64_t npair, OpMap Y, int64_t N, int64_t tilesM,
                                                            int64_t tilesN, int nsplit, int r0, int64_t rows,
                                                            double* part) {
  __shared__ double smem[2 * C::STAGE];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave % C::WM, wn = wave / C::WM;
  const int64_t ntile = tilesM * tilesN;
  // split major, then row band: the tiles of one P range sit on one XCD, and the column tiles
  // of a band side by side
  const int64_t item = xcd_remap(blockIdx.x, ntile * nsplit);
  const int split = (int)(item / ntile);
  const int64_t tile = item % ntile;
  const int m0 = r0 + (int)((tile / tilesN) * C::BM), n0 = (int)((tile % tilesN) * C::BN);
  const int64_t P0 = naux * split / nsplit, P1 = naux * (split + 1) / nsplit;
  const int nks = (nao + C::BK - 1) / C::BK;
  d4 acc[C::TM][C::TN];
  zero_acc<C>(acc);
  if (P1 > P0) {
    HalfSrc<C> src;
    src.Cm = &Y;
    src.c.init(Y, n0, 0, P0 * nks, P1 * nks, t);
    src.init(B, npair, P0, P1, nao, m0, t);
    mainloop<C>(src, smem, (P1 - P0) * nks, acc, wm, wn, lane);
  }
  const OutMap po = out_plain(part + (int64_t)split * rows * N, rows, N, N);
  store_tile<C, false>(po, 0, m0 - r0, n0, acc, wm, wn, lane);
}

// ---------------------------------------------------------------------------------------
// v[z][P] = sum_{m, c} C[z][m][c] w[z][c] X[P][m][z*nocc + c], one workgroup per (P, z),
// fixed-order reduction (deterministic).
__global__ void __launch_bounds__(256) jvec_kernel(const double* __restrict__ X, int64_t nao, int64_t ldx,
                                                   const double* __restrict__ Cm, const double* __restrict__ w,
                                                   int64_t nocc, double* __restrict__ v, int64_t ldv,
                                                   int accumulate) {
  __shared__ double red[4];
  const int64_t P = blockIdx.x, z = blockIdx.y;
  const double* Xp = X + P * nao * ldx + z * nocc;
  const double* Cz = Cm + z * nao * nocc;
  const double* wz = w ? w + z * nocc : nullptr;
  double s = 0.0;
  if (ldx == nocc && !wz) {
    // X_P and the factor are both contiguous [nao * nocc]: a dot product with four loads in flight
    const int64_t n = nao * nocc;
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t e = threadIdx.x;
    for (; e + 768 < n; e += 1024) {
      s = fma(Cz[e], Xp[e], s);
      s1 = fma(Cz[e + 256], Xp[e + 256], s1);
      s2 = fma(Cz[e + 512], Xp[e + 512], s2);
      s3 = fma(Cz[e + 768], Xp[e + 768], s3);
    }
    for (; e < n; e += 256) s = fma(Cz[e], Xp[e], s);
    s = (s + s1) + (s2 + s3);
  } else {
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
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    v[z * ldv + P] = accumulate ? v[z * ldv + P] + r : r;
  }
}

// J[z][i][j] = sum_P v[z][P] b^P_{ij}, streaming B once.  A workgroup owns kCoulombPairs * 256
// consecutive packed pairs (thread t the pairs t + 256 r) for every P, so each P row is read as
// runs of 8 KB; v is staged through LDS in blocks of 256 P.
constexpr int kCoulombZ = 4;
constexpr int kCoulombPairs = 4;
__global__ void __launch_bounds__(256) coulomb_kernel(const double* __restrict__ B, int64_t naux, int64_t nao,
                                                      int64_t npair, const double* __restrict__ v, int nz,
                                                      int64_t vstride, double* __restrict__ J, int64_t jstride,
                                                      int accumulate) {
  __shared__ double vs[kCoulombZ][256];
  const int64_t p0 = (int64_t)blockIdx.x * (256 * kCoulombPairs) + threadIdx.x;
  int64_t pc[kCoulombPairs];   // the pairs, clamped to the last one (read, never stored)
#pragma unroll
  for (int r = 0; r < kCoulombPairs; ++r) pc[r] = p0 + 256 * r < npair ? p0 + 256 * r : npair - 1;
  double acc[kCoulombPairs][kCoulombZ];
#pragma unroll
  for (int r = 0; r < kCoulombPairs; ++r)
#pragma unroll
    for (int z = 0; z < kCoulombZ; ++z) acc[r][z] = 0.0;
  for (int64_t P0 = 0; P0 < naux; P0 += 256) {
    const int64_t cnt = naux - P0 < 256 ? naux - P0 : 256;
    __syncthreads();
    for (int z = 0; z < nz; ++z) vs[z][threadIdx.x] = threadIdx.x < cnt ? v[z * vstride + P0 + threadIdx.x] : 0.0;
    __syncthreads();
    const double* Bp = B + P0 * npair;
#pragma unroll 2
    for (int q = 0; q < cnt; ++q) {
      double b[kCoulombPairs];
#pragma unroll
      for (int r = 0; r < kCoulombPairs; ++r) b[r] = Bp[(int64_t)q * npair + pc[r]];
#pragma unroll
      for (int z = 0; z < kCoulombZ; ++z) {
        if (z < nz) {
          const double w = vs[z][q];
#pragma unroll
          for (int r = 0; r < kCoulombPairs; ++r) acc[r][z] = fma(w, b[r], acc[r][z]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kCoulombPairs; ++r) {
    const int64_t p = p0 + 256 * r;
    if (p >= npair) break;
    int64_t i = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > p) --i;
    while ((i + 1) * (i + 2) / 2 <= p) ++i;
    const int64_t j = p - i * (i + 1) / 2;
    for (int z = 0; z < nz; ++z) {
      const double x = accumulate ? J[z * jstride + i * nao + j] + acc[r][z] : acc[r][z];   // J is symmetric
      J[z * jstride + i * nao + j] = x;
      J[z * jstride + j * nao + i] = x;
    }
  }
}

__global__ void __launch_bounds__(256) add_kernel(const double* __restrict__ x, int64_t n, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] += x[i];
}

// y[r][c] (+)= x[r][c] for a contiguous x [rows][cols] and y of row stride ldy
__global__ void __launch_bounds__(256) copy_rows_kernel(const double* __restrict__ x, int64_t rows, int64_t cols,
                                                        double* __restrict__ y, int64_t ldy, int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows * cols) return;
  double* d = y + (i / cols) * ldy + i % cols;
  *d = accumulate ? *d + x[i] : x[i];
}

__global__ void __launch_bounds__(256) scale_cols_kernel(const double* __restrict__ X, int64_t n, int64_t ncol,
                                                         const double* __restrict__ w, double* __restrict__ Xw) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) Xw[i] = X[i] * w[i % ncol];
}

// g[pair(i,j)] = G[i][j] + G[j][i] for i > j, G[i][i] on the diagonal
__global__ void __launch_bounds__(256) pair_weights_kernel(const double* __restrict__ G, int64_t nao,
                                                           double* __restrict__ g) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t npair = nao * (nao + 1) / 2;
  if (p >= npair) return;
  G += (int64_t)blockIdx.y * nao * nao;   // matrix blockIdx.y of a batch
  g += (int64_t)blockIdx.y * npair;
  int64_t i = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > p) --i;
  while ((i + 1) * (i + 2) / 2 <= p) ++i;
  const int64_t j = p - i * (i + 1) / 2;
  g[p] = i == j ? G[i * nao + i] : G[i * nao + j] + G[j * nao + i];
}

// u[P] = sum_pair B[P][pair] g[pair]: four rows of B per workgroup share each read of g; a
// fixed-order reduction keeps it deterministic.
constexpr int kJvRows = 4;
// Partial sums part[c][P] = sum_{pair in chunk c} B[P][pair] g[pair] for kJvRows rows per
// workgroup (grid x) and kJvChunks chunks of the pairs (grid y).  Each step a thread takes the
// pairs p + 256 u (u < 4) of every row: each row is read as runs of 8 KB per workgroup.
constexpr int kJvChunks = 8;
__global__ void __launch_bounds__(256) jvec_packed_kernel(const double* __restrict__ B, int64_t naux, int64_t npair,
                                                          const double* __restrict__ g, double* __restrict__ part) {
  __shared__ double red[kJvRows][4];
  const int64_t P0 = (int64_t)blockIdx.x * kJvRows;
  const int64_t c = blockIdx.y, chunk = (npair + kJvChunks - 1) / kJvChunks;
  const int64_t p0 = c * chunk, p1 = p0 + chunk < npair ? p0 + chunk : npair;
  const double* rows[kJvRows];   // rows past the end read the last one (never stored)
#pragma unroll
  for (int r = 0; r < kJvRows; ++r) rows[r] = B + (P0 + r < naux ? P0 + r : naux - 1) * npair;
  double s[kJvRows];
#pragma unroll
  for (int r = 0; r < kJvRows; ++r) s[r] = 0.0;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += 1024) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t q = p + 256 * u;
      const bool ok = q < p1;
      const int64_t qc = ok ? q : p1 - 1;
      const double gq = ok ? g[qc] : 0.0;
#pragma unroll
      for (int r = 0; r < kJvRows; ++r) s[r] = fma(rows[r][qc], gq, s[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < kJvRows; ++r) {
    double x = s[r];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    if ((threadIdx.x & 63) == 0) red[r][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x < kJvRows && P0 + threadIdx.x < naux) {
    const int r = threadIdx.x;
    part[c * naux + P0 + r] = (red[r][0] + red[r][1]) + (red[r][2] + red[r][3]);
  }
}

__global__ void __launch_bounds__(256) jvec_chunks_kernel(const double* __restrict__ part, int64_t naux,
                                                          double* __restrict__ u) {
  const int64_t P = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (P >= naux) return;
  double s = 0.0;
  for (int c = 0; c < kJvChunks; ++c) s += part[c * naux + P];
  u[P] = s;
}

// out[z] = in[z] + in[z]^T (in place allowed: each pair (i, j), i <= j, is handled by one thread)
__global__ void __launch_bounds__(256) symmetrize_kernel(const double* in, int64_t n, int64_t nz, double* out) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nn = n * n;
  if (idx >= nn * nz) return;
  const int64_t z = idx / nn, rem = idx % nn, i = rem / n, j = rem % n;
  if (i > j) return;
  const double* a = in + z * nn;
  const double s = a[i * n + j] + a[j * n + i];
  out[z * nn + i * n + j] = s;
  out[z * nn + j * n + i] = s;
}

__global__ void __launch_bounds__(256) unpack_sym_kernel(const double* __restrict__ Jp, int64_t nz, int64_t nao,
                                                         int64_t npair, double* __restrict__ J) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= nz * npair) return;
  const int64_t z = idx / npair, p = idx % npair;
  int64_t i = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > p) --i;
  while ((i + 1) * (i + 2) / 2 <= p) ++i;
  const int64_t j = p - i * (i + 1) / 2;
  const double x = Jp[idx];
  J[z * nao * nao + i * nao + j] = x;
  J[z * nao * nao + j * nao + i] = x;
}

__global__ void __launch_bounds__(256) pack_lower_kernel(const double* __restrict__ A, int64_t nz, int64_t n,
                                                         int64_t npair, double* __restrict__ Ap) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= nz * npair) return;
  const int64_t z = idx / npair, p = idx % npair;
  int64_t i = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while (i * (i + 1) / 2 > p) --i;
  while ((i + 1) * (i + 2) / 2 <= p) ++i;
  const int64_t j = p - i * (i + 1) / 2;
  Ap[idx] = A[z * n * n + i * n + j];
}

// Cholesky factor of one kb x kb diagonal block (kb <= kCholNB) of the metric, in LDS, and the
// inverse of that factor.  A (row stride lda) holds the block with the earlier blocks' updates
// already subtracted; its lower triangle is read.  Right-looking elimination: column j is scaled
// by 1 / sqrt(pivot), then the trailing lower triangle takes the rank-1 update.  The inverse is
// then found one column per thread by forward substitution: thread c keeps column c of L^-1 in
// row c of the LDS array (the upper triangle, which the factor does not use), and reads the
// factor from the strictly lower triangle and the diagonal from dg.  Outputs: the factor back to
// A (lower, the block's strictly upper part zeroed) and L^-1 to Linv [kCholNB][kCholNB] (lower,
// upper zeroed).  info: the first block (first != 0) writes 0; a block that meets a pivot that
// is not positive writes k0 + j + 1 unless info already holds an earlier one.  After such a
// pivot the block goes on with pivot 1 so that every wave finishes.
__global__ void __launch_bounds__(256) chol_block_kernel(double* __restrict__ A, int64_t lda, int kb,
                                                         double* __restrict__ Linv, int* info, int64_t k0,
                                                         int first) {
  __shared__ double S[kCholNB][kCholNB + 1];
  __shared__ double dg[kCholNB];
  __shared__ int bad;
  const int t = threadIdx.x;
  for (int idx = t; idx < kb * kb; idx += 256) {
    const int i = idx / kb, j = idx % kb;
    S[i][j] = j <= i ? A[i * lda + j] : 0.0;
  }
  if (t == 0) bad = -1;
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    const double d = S[j][j];
    const double sd = d > 0.0 ? sqrt(d) : 1.0;
    const double r = 1.0 / sd;
    __syncthreads();
    if (t == 0) {
      if (!(d > 0.0) && bad < 0) bad = j;
      dg[j] = sd;
    }
    for (int i = j + 1 + t; i < kb; i += 256) S[i][j] *= r;
    __syncthreads();
    // trailing lower triangle: lane t % 64 takes columns c = j + 1 + (t % 64) + 64 q, the four
    // wave-groups t / 64 take every fourth row i >= c
    for (int c = j + 1 + (t & 63); c < kb; c += 64) {
      const double lc = S[c][j];
      for (int i = c + (t >> 6); i < kb; i += 4) S[i][c] -= S[i][j] * lc;
    }
    __syncthreads();
  }
  if (t < kb) {
    const int c = t;
    S[c][c] = 1.0 / dg[c];
    for (int i = c + 1; i < kb; ++i) {
      double acc = 0.0;
      for (int j = c; j < i; ++j) acc += S[i][j] * S[c][j];
      S[c][i] = -acc / dg[i];
    }
  }
  __syncthreads();
  for (int idx = t; idx < kb * kb; idx += 256) {
    const int i = idx / kb, j = idx % kb;
    A[i * lda + j] = j < i ? S[i][j] : (j == i ? dg[i] : 0.0);
    Linv[i * kCholNB + j] = j <= i ? S[j][i] : 0.0;
  }
  if (t == 0) {
    int cur = first ? 0 : *info;
    if (cur == 0 && bad >= 0) cur = (int)(k0 + bad + 1);
    *info = cur;
  }
}

// A[i][j] = 0 for j > i, n x n
__global__ void __launch_bounds__(256) zero_upper_kernel(double* A, int64_t n) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n * n) return;
  if (idx % n > idx / n) A[idx] = 0.0;
}

__global__ void __launch_bounds__(256) fill_zero_kernel(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void __launch_bounds__(256) fill_zero_strided_kernel(double* p, int64_t nz, int64_t s_z, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n * nz) p[(i / n) * s_z + i % n] = 0.0;
}

// ---------------------------------------------------------------------------------------
// Launchers

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// A flat contraction pays where padding each kb block to whole slabs wastes more than 4% of the
// slabs (at 300 per block, 1.3%, the padded loads measured faster than the flat ones).
static bool flat_pays(const OpMap& o) { return o.kc_n >= 16 && cdiv(o.kc_n, 16) * 16 * 100 > o.kc_n * 104; }

// A flat contraction adds the step from one kb block to the next to the within-slab offsets.
static bool flat_fits(const OpMap& o) {
  if (o.rows <= 0 || o.kc_n <= 0) return true;
  const int64_t last = o.rows - 1;
  const int64_t rh = o.s_rh ? last / o.rl : 0, rlo = o.s_rh ? o.rl - 1 : last;
  const int64_t top = rh * o.s_rh + rlo * o.s_rlo + 15 * o.s_kc + (o.s_kb - o.kc_n * o.s_kc);
  return o.s_kb >= o.kc_n * o.s_kc && top < (1LL << 32);
}

bool offsets_fit(const OpMap& o) {
  if (o.rows <= 0 || o.kc_n <= 0) return true;
  const int64_t last = o.rows - 1;
  const int64_t rh = o.s_rh ? last / o.rl : 0, rlo = o.s_rh ? o.rl - 1 : last;
  const int64_t kmax = o.kc_n - 1 + 15;   // a slab may address up to 15 entries past the end before clamping
  const int64_t top = rh * o.s_rh + rlo * o.s_rlo + kmax * o.s_kc;
  return o.rows < (1LL << 31) && o.rl < (1LL << 31) && top < (1LL << 32);
}

// Column tile of the half transform on one row of waves: the widest of {176, 96, 48} whose padded
// width is within 8% of the least padded one.  A wider tile reads each band of b^P fewer times
// per column, which outweighs a few percent of padded columns (at 1200 columns: 176 pads to
// 1232, 48 to 1200).
int half_tile_n(int64_t ncol) {
  const int cands[3] = {176, 96, 48};
  int64_t least = INT64_MAX;
  for (int c : cands) least = std::min<int64_t>(least, cdiv(ncol, c) * c);
  for (int c : cands)
    if (cdiv(ncol, c) * c * 100 <= least * 108) return c;
  return cands[2];
}

// Tilings of the half transform.  One row of waves (4 x 1 waves of 1 x 11, 2 x 6 or 2 x 3 MFMA
// blocks: 64 x 176, 128 x 96, 128 x 48) fits odd column counts (176 = 11 x 16), but its waves
// issue one LDS read per MFMA.  2 x 2 waves of 4 x 4 blocks read half as much per MFMA and keep
// the matrix cores busier (0.81 of the time against 0.73 for 1 x 11, both measured at N_ao =
// 1200), at 128-row bands and 128-column tiles.  The 2-D tiling takes the columns in 128-wide
// tiles plus one narrower remainder (96 or 64 wide: 2 x 2 waves of 4 x 3 or 4 x 2 blocks), the
// rows in whole 128-row bands, and the rows past the last whole band (if any) on one row of
// waves.  Each piece is a launch of its own; the choice is the tiling of least estimated time,
// padded area over the matrix-core busy fraction of its tile shape.
enum HalfCfg { kH176, kH96, kH48, kQ128, kQ96, kQ64 };
struct HalfSeg {
  int cfg;
  int64_t r0, r1, c0, c1;   // rows [r0, r1) and columns [c0, c1) of the output
};
static int half_cfg_rows(int cfg) { return cfg == kH176 ? 64 : 128; }
static int half_cfg_cols(int cfg) {
  switch (cfg) {
    case kH176: return 176;
    case kH96: return 96;
    case kH48: return 48;
    case kQ128: return 128;
    case kQ96: return 96;
    default: return 64;
  }
}
// matrix-core busy fraction of each tile shape (1 x 11 and 4 x 4 measured; the others estimated
// from their LDS reads per MFMA)
static double half_cfg_busy(int cfg) {
  switch (cfg) {
    case kH176: return 0.73;
    case kH96: return 0.72;
    case kH48: return 0.68;
    case kQ128: return 0.81;
    case kQ96: return 0.78;
    default: return 0.72;
  }
}
static double half_seg_cost(const HalfSeg& g) {
  const int bm = half_cfg_rows(g.cfg), bn = half_cfg_cols(g.cfg);
  return (double)(cdiv(g.r1 - g.r0, bm) * bm) * (double)(cdiv(g.c1 - g.c0, bn) * bn) / half_cfg_busy(g.cfg);
}
static int half_cfg_1d(int64_t ncol) {
  const int n = half_tile_n(ncol);
  return n == 176 ? kH176 : n == 96 ? kH96 : kH48;
}

// The pieces of the half transform of nao rows and ncol columns (at most 3).  `split_cols` says
// whether the output map can be cut along its columns (no column blocking).
static int half_scheme(int64_t nao, int64_t ncol, bool split_cols, HalfSeg* seg) {
  seg[0] = HalfSeg{half_cfg_1d(ncol), 0, nao, 0, ncol};
  if (!split_cols || nao < 128 || ncol < 64) return 1;
  double best = half_seg_cost(seg[0]);
  int nbest = 1;
  HalfSeg cand[3];
  for (int tail = 0; tail < 2; ++tail) {
    const int64_t rq = tail ? nao / 128 * 128 : nao;
    if (tail && (rq == nao || rq == 0)) continue;
    int n = 0;
    const int64_t cq = ncol / 128 * 128, rem = ncol - cq;
    if (cq > 0) cand[n++] = HalfSeg{kQ128, 0, rq, 0, cq};
    if (rem > 0) {   // the remainder columns on the cheapest tile of 128 rows
      const int rc[5] = {kQ128, kQ96, kQ64, kH96, kH48};
      double rbest = 0.0;
      for (int q = 0; q < 5; ++q) {
        const HalfSeg g{rc[q], 0, rq, cq, ncol};
        if (q == 0 || half_seg_cost(g) < rbest) {
          rbest = half_seg_cost(g);
          cand[n] = g;
        }
      }
      ++n;
    }
    if (tail) cand[n++] = HalfSeg{half_cfg_1d(ncol), rq, nao, 0, ncol};
    double cost = 0.0;
    for (int i = 0; i < n; ++i) cost += half_seg_cost(cand[i]);
    if (cost < best) {
      best = cost;
      nbest = n;
      for (int i = 0; i < n; ++i) seg[i] = cand[i];
    }
  }
  return nbest;
}

// `o` restricted to columns [c0, c1) (no column blocking: s_nh == 0)
static OutMap out_cols(OutMap o, int64_t c0, int64_t c1) {
  if (c0 < o.nsplit) {
    o.p += c0 * o.s_nl;
    o.nsplit -= c0;
  } else {
    o.p2 += c0 - o.nsplit;
    o.nsplit = 0;
  }
  o.N = std::min(o.N, c1) - c0;
  return o;
}

template <class Cg>
static hipError_t half_seg_go(const double* B, int64_t naux, int64_t nao, const double* C, int64_t ldc,
                              const HalfSeg& g, const OutMap& out, const JvEpi* jv, hipStream_t s) {
  const OpMap cm = op_map(C + g.c0, g.c1 - g.c0, 1, nao, ldc);
  const OutMap o = out_cols(out, g.c0, g.c1);
  const int64_t tm = cdiv(g.r1 - g.r0, Cg::BM), tn = cdiv(g.c1 - g.c0, Cg::BN);
  const int64_t nblk = tm * tn * naux;
  if (nblk == 0) return hipSuccess;
  if (nblk > 0x7fffffffLL || !offsets_fit(cm)) return hipErrorInvalidValue;
  const int64_t npair = nao * (nao + 1) / 2;
  if (jv) {
    if (o.alpha != 1.0 || o.accumulate) return hipErrorInvalidValue;
    JvEpi j = *jv;
    j.C = jv->C + g.c0;
    j.nv = (int)std::max<int64_t>(0, std::min<int64_t>(jv->nv - g.c0, g.c1 - g.c0));
    half_jv_kernel<Cg><<<dim3((unsigned)nblk), dim3(Cg::NT), 0, s>>>(B, naux, (int)nao, npair, cm, o, tm, tn,
                                                                     (int)g.r0, j);
  } else if (o.alpha != 1.0 || o.accumulate) {
    half_kernel<Cg, true><<<dim3((unsigned)nblk), dim3(Cg::NT), 0, s>>>(B, naux, (int)nao, npair, cm, o, tm, tn,
                                                                       (int)g.r0);
  } else {
    half_kernel<Cg, false><<<dim3((unsigned)nblk), dim3(Cg::NT), 0, s>>>(B, naux, (int)nao, npair, cm, o, tm, tn,
                                                                        (int)g.r0);
  }
  return hipGetLastError();
}

static int64_t half_seg_tiles(const HalfSeg& g) {
  return cdiv(g.r1 - g.r0, half_cfg_rows(g.cfg)) * cdiv(g.c1 - g.c0, half_cfg_cols(g.cfg));
}

// Two pieces on the same rows, 128-wide tiles on columns [0, cq) and one tile of CB on the rest,
// as one launch (half_pair_kernel).
template <class CB>
static hipError_t half_pair_go(const double* B, int64_t naux, int64_t nao, const double* C, int64_t ldc,
                               int64_t ncol, const HalfSeg& a, const OutMap& out, JvEpi* jv, hipStream_t s) {
  const OpMap cm = op_map(C, ncol, 1, nao, ldc);
  const int64_t tm = cdiv(a.r1 - a.r0, CfgQ128::BM), nA = a.c1 / CfgQ128::BN;
  const int64_t nblk = tm * (nA + 1) * naux;
  if (nblk == 0) return hipSuccess;
  if (nblk > 0x7fffffffLL || !offsets_fit(cm)) return hipErrorInvalidValue;
  const int64_t npair = nao * (nao + 1) / 2;
  const JvEpi j = jv ? *jv : JvEpi{};
  const dim3 g((unsigned)nblk);
  if (jv) {
    if (out.alpha != 1.0 || out.accumulate) return hipErrorInvalidValue;
    half_pair_kernel<CfgQ128, CB, false, true><<<g, CfgQ128::NT, 0, s>>>(B, naux, (int)nao, npair, cm, out, tm, nA,
                                                                          (int)a.r0, j);
  } else if (out.alpha != 1.0 || out.accumulate) {
    half_pair_kernel<CfgQ128, CB, true, false><<<g, CfgQ128::NT, 0, s>>>(B, naux, (int)nao, npair, cm, out, tm, nA,
                                                                          (int)a.r0, j);
  } else {
    half_pair_kernel<CfgQ128, CB, false, false><<<g, CfgQ128::NT, 0, s>>>(B, naux, (int)nao, npair, cm, out, tm, nA,
                                                                           (int)a.r0, j);
  }
  return hipGetLastError();
}

static hipError_t half_run(const double* B, int64_t naux, int64_t nao, const double* C, int64_t ldc, int64_t ncol,
                           const OutMap& out, JvEpi* jv, hipStream_t s) {
  HalfSeg seg[3];
  const int n = half_scheme(nao, ncol, out.s_nh == 0, seg);
  if (jv) {
    jv->T = 0;
    for (int i = 0; i < n; ++i) jv->T += half_seg_tiles(seg[i]);
    jv->toff = 0;
  }
  for (int i = 0; i < n; ++i) {
    // 128-wide tiles from column 0 and a one-tile remainder on the same rows: one launch
    if (i + 1 < n && seg[i].cfg == kQ128 && seg[i].c0 == 0 && seg[i].c1 % CfgQ128::BN == 0 &&
        seg[i + 1].r0 == seg[i].r0 && seg[i + 1].r1 == seg[i].r1 && seg[i + 1].c0 == seg[i].c1 &&
        seg[i + 1].c1 - seg[i + 1].c0 <= half_cfg_cols(seg[i + 1].cfg) && half_cfg_rows(seg[i + 1].cfg) == 128) {
      hipError_t e;
      switch (seg[i + 1].cfg) {
        case kQ128: e = half_pair_go<CfgQ128>(B, naux, nao, C, ldc, ncol, seg[i], out, jv, s); break;
        case kQ96: e = half_pair_go<CfgQ96>(B, naux, nao, C, ldc, ncol, seg[i], out, jv, s); break;
        case kQ64: e = half_pair_go<CfgQ64>(B, naux, nao, C, ldc, ncol, seg[i], out, jv, s); break;
        case kH96: e = half_pair_go<CfgH96>(B, naux, nao, C, ldc, ncol, seg[i], out, jv, s); break;
        default: e = half_pair_go<CfgH48>(B, naux, nao, C, ldc, ncol, seg[i], out, jv, s); break;
      }
      if (e != hipSuccess) return e;
      if (jv) jv->toff += half_seg_tiles(seg[i]) + half_seg_tiles(seg[i + 1]);
      ++i;
      continue;
    }
    hipError_t e;
    switch (seg[i].cfg) {
      case kH176: e = half_seg_go<CfgH176>(B, naux, nao, C, ldc, seg[i], out, jv, s); break;
      case kH96: e = half_seg_go<CfgH96>(B, naux, nao, C, ldc, seg[i], out, jv, s); break;
      case kH48: e = half_seg_go<CfgH48>(B, naux, nao, C, ldc, seg[i], out, jv, s); break;
      case kQ128: e = half_seg_go<CfgQ128>(B, naux, nao, C, ldc, seg[i], out, jv, s); break;
      case kQ96: e = half_seg_go<CfgQ96>(B, naux, nao, C, ldc, seg[i], out, jv, s); break;
      default: e = half_seg_go<CfgQ64>(B, naux, nao, C, ldc, seg[i], out, jv, s); break;
    }
    if (e != hipSuccess) return e;
    if (jv) jv->toff += half_seg_tiles(seg[i]);
  }
  return hipSuccess;
}

hipError_t launch_half_transform(const double* B, int64_t naux, int64_t nao, const double* C, int64_t ldc,
                                 int64_t ncol, const OutMap& out, hipStream_t s) {
  return half_run(B, naux, nao, C, ldc, ncol, out, nullptr, s);
}

int64_t half_tiles(int64_t nao, int64_t ncol) {
  HalfSeg seg[3];
  const int n = half_scheme(nao, ncol, true, seg);
  int64_t T = 0;
  for (int i = 0; i < n; ++i) T += half_seg_tiles(seg[i]);
  return T;
}

hipError_t launch_half_transform_jvec(const double* B, int64_t naux, int64_t nao, const double* C, int64_t ldc,
                                      int64_t ncol, const OutMap& out, const double* w, int64_t nv, double* part,
                                      double* v, int accumulate, hipStream_t s) {
  if (nv < 0 || nv > ncol || nv > 0x7fffffffLL || out.s_nh != 0) return hipErrorInvalidValue;
  if (naux == 0) return hipSuccess;
  JvEpi jv{C, ldc, w, (int)nv, part, 0, 0};
  hipError_t e = half_run(B, naux, nao, C, ldc, ncol, out, &jv, s);
  if (e != hipSuccess) return e;
  if (jv.T == 0) return hipErrorInvalidValue;
  jv_reduce_kernel<<<(unsigned)cdiv(naux, 256), 256, 0, s>>>(part, jv.T, naux, v, accumulate);
  return hipGetLastError();
}

// The 256-row tile when it pads the rows no more than the 128-row one.
static bool gemm_tall(int64_t M) {
  return M >= 256 && cdiv(M, CfgTall::BM) * CfgTall::BM <= cdiv(M, CfgSq::BM) * CfgSq::BM;
}

template <class Cg, bool GEN, bool CLAMP>
static void gemm_go(const OpMap& A, const OpMap& Bm, const OutMap& O, dim3 grid, int64_t tm, int64_t tn, double* part,
                    hipStream_t s) {
  const bool ak = A.s_kc == 1, bk = Bm.s_kc == 1;
  if (ak && bk) gemm_kernel<Cg, true, true, GEN, CLAMP><<<grid, Cg::NT, 0, s>>>(A, Bm, O, tm, tn, part);
  else if (ak) gemm_kernel<Cg, true, false, GEN, CLAMP><<<grid, Cg::NT, 0, s>>>(A, Bm, O, tm, tn, part);
  else if (bk) gemm_kernel<Cg, false, true, GEN, CLAMP><<<grid, Cg::NT, 0, s>>>(A, Bm, O, tm, tn, part);
  else gemm_kernel<Cg, false, false, GEN, CLAMP><<<grid, Cg::NT, 0, s>>>(A, Bm, O, tm, tn, part);
}

template <class Cg>
static hipError_t gemm_launch_cfg(const OpMap& A, const OpMap& Bm, const OutMap& O, int64_t nz, int nsplit,
                                  double* part, hipStream_t s) {
  const int64_t tm = cdiv(O.M, Cg::BM), tn = cdiv(O.N, Cg::BN);
  if (tm * tn == 0 || nz == 0) return hipSuccess;
  if (tm * tn > 0x7fffffffLL || nz > 65535 || nsplit < 1 || nsplit > 65535 || !offsets_fit(A) || !offsets_fit(Bm) ||
      A.kc_n != Bm.kc_n || A.kb_n != Bm.kb_n)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)(tm * tn), (unsigned)nsplit, (unsigned)nz);
  // whole slabs (no clamping) when the contraction chunks are multiples of 16
  const bool clamp = A.kc_n % 16 != 0;
  if (!part && (O.alpha != 1.0 || O.accumulate)) gemm_go<Cg, true, true>(A, Bm, O, grid, tm, tn, part, s);
  else if (clamp) gemm_go<Cg, false, true>(A, Bm, O, grid, tm, tn, part, s);
  else gemm_go<Cg, false, false>(A, Bm, O, grid, tm, tn, part, s);
  return hipGetLastError();
}

static hipError_t gemm_launch(const OpMap& A, const OpMap& Bm, const OutMap& O, int64_t nz, int nsplit,
                              double* part, hipStream_t s) {
  const int64_t rem = O.M % CfgSq::BM, tn = cdiv(O.N, CfgSq::BN);
  if (gemm_tall(O.M) && rem > 0 && rem <= CfgRowTail::BM && nz == 1 && nsplit == 1 && !part && O.alpha == 1.0 &&
      !O.accumulate && A.kc_n % 16 == 0 && (O.M / CfgSq::BM + 1) * tn <= 0x7fffffffLL && offsets_fit(A) &&
      offsets_fit(Bm) && A.kc_n == Bm.kc_n && A.kb_n == Bm.kb_n) {
    const int64_t nband = O.M / CfgSq::BM;
    const dim3 grid((unsigned)((nband + 1) * tn));
    const bool ak = A.s_kc == 1, bk = Bm.s_kc == 1;
    if (ak && bk) gemm_tail_kernel<true, true><<<grid, CfgSq::NT, 0, s>>>(A, Bm, O, nband, tn);
    else if (ak) gemm_tail_kernel<true, false><<<grid, CfgSq::NT, 0, s>>>(A, Bm, O, nband, tn);
    else if (bk) gemm_tail_kernel<false, true><<<grid, CfgSq::NT, 0, s>>>(A, Bm, O, nband, tn);
    else gemm_tail_kernel<false, false><<<grid, CfgSq::NT, 0, s>>>(A, Bm, O, nband, tn);
    return hipGetLastError();
  }
  return gemm_tall(O.M) ? gemm_launch_cfg<CfgTall>(A, Bm, O, nz, nsplit, part, s)
                        : gemm_launch_cfg<CfgSq>(A, Bm, O, nz, nsplit, part, s);
}

hipError_t launch_gemm(const OpMap& A, const OpMap& Bm, const OutMap& O, int64_t nz, hipStream_t s) {
  return gemm_launch(A, Bm, O, nz, 1, nullptr, s);
}

int64_t gemm_slabs(const OpMap& A) { return A.kb_n * cdiv(A.kc_n, 16); }

// Workgroups resident at once for the MFMA kernels on MI355X: 256 CUs x 2 (each kernel is sized
// for two workgroups per CU).  A launch of W equal workgroups takes ceil(W / kResident) rounds.
static constexpr int64_t kResident = 512;

// Split count s in [1, max_split] for a launch of tiles * s equal workgroups: the one that fills
// its last round best, among counts that fill at least one round (when any does), the smaller
// on ties (less partial-sum traffic).
static int balanced_splits(int64_t tiles, int64_t max_split) {
  if (tiles <= 0) return 1;
  if (max_split < 1) max_split = 1;
  if (max_split > 4096) max_split = 4096;
  const int64_t s_fill = cdiv(kResident, tiles);
  int64_t lo = s_fill <= max_split ? s_fill : max_split, hi = 4 * lo < max_split ? 4 * lo : max_split;
  if (hi < lo) hi = lo;
  int best = (int)lo;
  double best_eff = -1.0;
  for (int64_t sp = lo; sp <= hi; ++sp) {
    const int64_t w = tiles * sp;
    const double eff = (double)w / (double)(cdiv(w, kResident) * kResident);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = (int)sp;
    }
  }
  return best;
}

// balanced_splits(tiles, m) for any m <= max_split is at most this: its search runs over
// [lo, 4 lo] with lo <= kResident / tiles rounded up, and never past max_split.
static int balanced_splits_bound(int64_t tiles, int64_t max_split) {
  if (tiles <= 0 || max_split < 1) return 1;
  const int64_t b = 4 * cdiv(kResident, tiles);
  return (int)(max_split < b ? max_split : b);
}

int gemm_splits_bound(int64_t M, int64_t N, int64_t nslab) {
  if (gemm_tall(M)) return balanced_splits_bound(2 * cdiv(M, CfgTall::BM) * cdiv(N, CfgTall::BN), nslab / 4);
  return balanced_splits_bound(cdiv(M, CfgSq::BM) * cdiv(N, CfgSq::BN), nslab / 4);
}

int gemm_splits(int64_t M, int64_t N, int64_t nslab) {
  // at least four slabs per split; a tall tile takes the room of two resident workgroups
  if (gemm_tall(M)) return balanced_splits(2 * cdiv(M, CfgTall::BM) * cdiv(N, CfgTall::BN), nslab / 4);
  return balanced_splits(cdiv(M, CfgSq::BM) * cdiv(N, CfgSq::BN), nslab / 4);
}

hipError_t launch_split_reduce(const double* part, int nsplit, const OutMap& O, hipStream_t s) {
  const int64_t MN = O.M * O.N;
  if (MN == 0) return hipSuccess;
  split_reduce_kernel<<<(unsigned)cdiv(MN, 256), 256, 0, s>>>(part, nsplit, O);
  return hipGetLastError();
}

hipError_t launch_gemm_split(const OpMap& A, const OpMap& Bm, const OutMap& O, int nsplit, double* part,
                             hipStream_t s) {
  if (nsplit <= 1) return gemm_launch(A, Bm, O, 1, 1, nullptr, s);
  hipError_t e = gemm_launch(A, Bm, O, 1, nsplit, part, s);
  if (e != hipSuccess) return e;
  const int64_t MN = O.M * O.N;
  if (MN == 0) return hipSuccess;
  split_reduce_kernel<<<(unsigned)cdiv(MN, 256), 256, 0, s>>>(part, nsplit, O);
  return hipGetLastError();
}

// The P-summed packed product takes the half transform's tilings (half_scheme): each piece is a
// launch of its own with its own P split (filling the resident workgroups) and its own partials
// [splits][rows][cols], reduced into O piece by piece.
static int half_reduce_seg_splits(const HalfSeg& g, int64_t naux) { return balanced_splits(half_seg_tiles(g), naux); }

int64_t half_reduce_part_bound(int64_t nao, int64_t N, int64_t naux) {
  HalfSeg seg[3];
  const int n = half_scheme(nao, N, true, seg);
  int64_t total = 0;
  for (int i = 0; i < n; ++i)
    total += (int64_t)balanced_splits_bound(half_seg_tiles(seg[i]), naux) * (seg[i].r1 - seg[i].r0) *
             (seg[i].c1 - seg[i].c0);
  return total;
}

template <class Cg>
static hipError_t half_reduce_go(const double* B, int64_t naux, int64_t nao, const OpMap& Y, const HalfSeg& g,
                                 int nsplit, double* part, hipStream_t s) {
  OpMap Yg = Y;
  Yg.p = Y.p + g.c0;
  Yg.rows = Yg.rl = g.c1 - g.c0;
  const int64_t tm = cdiv(g.r1 - g.r0, Cg::BM), tn = cdiv(g.c1 - g.c0, Cg::BN);
  const int64_t nblk = tm * tn * nsplit;
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  half_reduce_kernel<Cg><<<dim3((unsigned)nblk), Cg::NT, 0, s>>>(B, naux, (int)nao, nao * (nao + 1) / 2, Yg,
                                                                g.c1 - g.c0, tm, tn, nsplit, (int)g.r0,
                                                                g.r1 - g.r0, part);
  return hipGetLastError();
}

hipError_t launch_half_reduce(const double* B, int64_t naux, int64_t nao, const OpMap& Y, const OutMap& O,
                              double* part, hipStream_t s) {
  if (nao <= 0 || O.N <= 0) return hipSuccess;
  if (naux < 1 || !offsets_fit(Y) || O.s_nh != 0 || O.s_mh != 0) return hipErrorInvalidValue;
  HalfSeg seg[3];
  const int n = half_scheme(nao, O.N, true, seg);
  for (int i = 0; i < n; ++i) {
    const HalfSeg& g = seg[i];
    const int ns = half_reduce_seg_splits(g, naux);
    hipError_t e;
    switch (g.cfg) {
      case kH176: e = half_reduce_go<CfgH176>(B, naux, nao, Y, g, ns, part, s); break;
      case kH96: e = half_reduce_go<CfgH96>(B, naux, nao, Y, g, ns, part, s); break;
      case kH48: e = half_reduce_go<CfgH48>(B, naux, nao, Y, g, ns, part, s); break;
      case kQ128: e = half_reduce_go<CfgQ128>(B, naux, nao, Y, g, ns, part, s); break;
      case kQ96: e = half_reduce_go<CfgQ96>(B, naux, nao, Y, g, ns, part, s); break;
      default: e = half_reduce_go<CfgQ64>(B, naux, nao, Y, g, ns, part, s); break;
    }
    if (e != hipSuccess) return e;
    // the piece's rows and columns of O
    OutMap Oc = out_cols(O, g.c0, g.c1);
    if (Oc.nsplit > 0) Oc.p += g.r0 * Oc.s_ml;
    if (Oc.p2) Oc.p2 += g.r0 * Oc.s2_m;
    Oc.M = g.r1 - g.r0;
    const int64_t MN = Oc.M * Oc.N;
    split_reduce_kernel<<<(unsigned)cdiv(MN, 256), 256, 0, s>>>(part, ns, Oc);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    part += (int64_t)ns * MN;
  }
  return hipSuccess;
}

hipError_t launch_pair_weights(const double* G, int64_t nao, double* g, hipStream_t s) {
  const int64_t npair = nao * (nao + 1) / 2;
  if (npair == 0) return hipSuccess;
  pair_weights_kernel<<<(unsigned)cdiv(npair, 256), 256, 0, s>>>(G, nao, g);
  return hipGetLastError();
}

hipError_t launch_dens_pairs(const double* C, int64_t nao, int64_t nocc, int64_t ndm, double* D, double* Dw,
                             hipStream_t s) {
  const int64_t npair = nao * (nao + 1) / 2;
  if (npair == 0 || ndm == 0) return hipSuccess;
  if (ndm > 65535) return hipErrorInvalidValue;
  // D_z = C_z C_z^T on the matrix cores, then packed with the pair weights
  OpMap Cz = op_map(C, nao, nocc, nocc, 1);
  Cz.s_z = nao * nocc;
  OutMap O = out_plain(D, nao, nao, nao);
  O.s_z = nao * nao;
  hipError_t e = launch_gemm(Cz, Cz, O, ndm, s);
  if (e != hipSuccess) return e;
  pair_weights_kernel<<<dim3((unsigned)cdiv(npair, 256), (unsigned)ndm), 256, 0, s>>>(D, nao, Dw);
  return hipGetLastError();
}

int jvec_packed_chunks() { return kJvChunks; }

hipError_t launch_jvec_packed(const double* B, int64_t naux, int64_t nao, const double* g, double* part, double* u,
                              hipStream_t s) {
  if (naux == 0) return hipSuccess;
  jvec_packed_kernel<<<dim3((unsigned)cdiv(naux, kJvRows), kJvChunks), 256, 0, s>>>(B, naux, nao * (nao + 1) / 2, g,
                                                                                    part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  jvec_chunks_kernel<<<(unsigned)cdiv(naux, 256), 256, 0, s>>>(part, naux, u);
  return hipGetLastError();
}

hipError_t launch_symmetrize(const double* in, int64_t n, int64_t nz, double* out, hipStream_t s) {
  const int64_t tot = n * n * nz;
  if (tot == 0) return hipSuccess;
  symmetrize_kernel<<<(unsigned)cdiv(tot, 256), 256, 0, s>>>(in, n, nz, out);
  return hipGetLastError();
}



int syrk_tile_for(int64_t n) { return n <= 640 ? CfgSyrk64::BM : CfgSyrk::BM; }

int syrk_splits(int64_t n, int64_t kb_n, int64_t nz) {
  const int64_t T = cdiv(n, syrk_tile_for(n));
  return balanced_splits(T * (T + 1) / 2 * (nz > 0 ? nz : 1), kb_n);
}

int syrk_splits_bound(int64_t n, int64_t kb_n, int64_t nz) {
  const int64_t T = cdiv(n, syrk_tile_for(n));
  return balanced_splits_bound(T * (T + 1) / 2 * (nz > 0 ? nz : 1), kb_n < 4096 ? kb_n : 4096);
}

template <class Cg>
static hipError_t syrk_go(const OpMap& A, const OpMap& Bw, int64_t n, int64_t nz, int nsplit, double* Kpart,
                          hipStream_t s) {
  const int64_t T = cdiv(n, Cg::BM);
  const int64_t npairs = T * (T + 1) / 2;
  if (npairs == 0 || nz == 0) return hipSuccess;
  if (nz > 65535 || !offsets_fit(A)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(npairs * nsplit), 1, (unsigned)nz);
  const bool clamp = A.kc_n % 16 != 0;
  // contraction chunks that are not whole slabs: one flat contraction (no padded slabs) unless
  // weighted or shorter than a slab
  const bool flat = clamp && !Bw.ks && flat_pays(A) && flat_fits(A);
  // weighted: the clamping loader in every case (without it the weighted 128-wide tiles need more
  // than 256 registers per lane and run one wave per SIMD)
  if (Bw.ks) syrk_kernel<Cg, true, true><<<grid, Cg::NT, 0, s>>>(A, Bw, n, nz, nsplit, npairs, Kpart);
  else if (flat) syrk_kernel<Cg, false, false, true><<<grid, Cg::NT, 0, s>>>(A, Bw, n, nz, nsplit, npairs, Kpart);
  else if (clamp) syrk_kernel<Cg, false, true><<<grid, Cg::NT, 0, s>>>(A, Bw, n, nz, nsplit, npairs, Kpart);
  else syrk_kernel<Cg, false, false><<<grid, Cg::NT, 0, s>>>(A, Bw, n, nz, nsplit, npairs, Kpart);
  return hipGetLastError();
}

hipError_t launch_syrk_partial(const OpMap& A, const OpMap& Bw, int64_t n, int64_t nz, int nsplit, double* Kpart,
                               hipStream_t s) {
  return syrk_tile_for(n) == CfgSyrk64::BM ? syrk_go<CfgSyrk64>(A, Bw, n, nz, nsplit, Kpart, s)
                                           : syrk_go<CfgSyrk>(A, Bw, n, nz, nsplit, Kpart, s);
}

// ---- grouped launches ----
// Cuts items [0, start[n]) into 8 contiguous chunks of about equal cost (each item of problem p
// costs cost[p]) and returns the length of the longest (the grid is 8 times that).
static int64_t xcd_chunks(const int64_t* start, const double* cost, int n, int64_t* xs) {
  double total = 0.0;
  for (int p = 0; p < n; ++p) total += (double)(start[p + 1] - start[p]) * cost[p];
  xs[0] = 0;
  int p = 0;
  double before = 0.0;   // cost of the items of problems before p
  for (int x = 1; x < 8; ++x) {
    const double target = total * x / 8.0;
    while (p < n && before + (double)(start[p + 1] - start[p]) * cost[p] <= target) {
      before += (double)(start[p + 1] - start[p]) * cost[p];
      ++p;
    }
    int64_t i = start[n];
    if (p < n) {
      i = start[p] + (int64_t)((target - before) / cost[p] + 0.5);
      if (i > start[p + 1]) i = start[p + 1];
    }
    xs[x] = i < xs[x - 1] ? xs[x - 1] : i;
  }
  xs[8] = start[n];
  int64_t longest = 1;
  for (int x = 0; x < 8; ++x) longest = xs[x + 1] - xs[x] > longest ? xs[x + 1] - xs[x] : longest;
  return longest;
}

// rows [r0[p], r1[p]) of problem p (all rows when r0 is null); problems with no rows are skipped
template <class Cg>
static hipError_t half_group_go(const GroupHalf* probs, int n, hipStream_t s, const int64_t* r0 = nullptr,
                                const int64_t* r1 = nullptr) {
  HalfGroup g{};
  g.start[0] = 0;
  for (int i = 0; i < n; ++i) {
    const GroupHalf& q = probs[i];
    const int64_t a = r0 ? r0[i] : 0, b = r1 ? r1[i] : q.nao;
    if (b <= a) continue;
    const int p = g.n++;
    HalfDesc& d = g.d[p];
    d.B = q.B;
    d.nao = (int)q.nao;
    d.r0 = (int)a;
    d.npair = q.nao * (q.nao + 1) / 2;
    d.Cm = op_map(q.C, q.ncol, 1, q.nao, q.ldc);
    d.out = q.out;
    d.tilesM = cdiv(b - a, Cg::BM);
    d.tilesN = cdiv(q.ncol, Cg::BN);
    if (!offsets_fit(d.Cm) || q.out.alpha != 1.0 || q.out.accumulate) return hipErrorInvalidValue;
    g.start[p + 1] = g.start[p] + d.tilesM * d.tilesN * q.naux;
  }
  if (g.n == 0 || g.start[g.n] == 0) return hipSuccess;
  if (g.start[g.n] > 0x7fffffffLL) return hipErrorInvalidValue;
  double cost[kMaxGroup];   // slabs per item, plus about two for the prologue and the epilogue
  for (int p = 0; p < g.n; ++p) cost[p] = (double)cdiv(g.d[p].nao, Cg::BK) + 2.0;
  const int64_t per = xcd_chunks(g.start, cost, g.n, g.xs);
  if (8 * per > 0x7fffffffLL) return hipErrorInvalidValue;
  half_group_kernel<Cg><<<(unsigned)(8 * per), Cg::NT, 0, s>>>(g);
  return hipGetLastError();
}

// The 2-D tiling of a problem in a group: the cheaper (padded area over matrix-core busy
// fraction, as in half_scheme) of all rows on 128 x 128 tiles and the whole 128-row bands on them
// with the rest of the rows on 64 x 176 tiles.  Returns the rows on 128 x 128 tiles and the cost.
static int64_t half_group_2d_rows(int64_t nao, int64_t ncol, double* cost) {
  const int64_t rq = nao / 128 * 128;
  const double all = half_seg_cost(HalfSeg{kQ128, 0, nao, 0, ncol});
  const double split = rq > 0 && rq < nao ? half_seg_cost(HalfSeg{kQ128, 0, rq, 0, ncol}) +
                                                 half_seg_cost(HalfSeg{kH176, rq, nao, 0, ncol})
                                           : all;
  *cost = std::min(all, split);
  return split < all ? rq : nao;
}

int half_group_tile_for(const int64_t* nao, const int64_t* ncol, int n) {
  double c2 = 0.0, c1 = 0.0, c;
  for (int i = 0; i < n; ++i) {
    half_group_2d_rows(nao[i], ncol[i], &c);
    c2 += c * (double)nao[i];   // the contraction runs over nao
    c1 += half_seg_cost(HalfSeg{kH176, 0, nao[i], 0, ncol[i]}) * (double)nao[i];
  }
  return c2 < c1 ? 128 : 176;
}

static hipError_t half_group_2d(const GroupHalf* probs, int n, hipStream_t s) {
  int64_t q0[kMaxGroup], q1[kMaxGroup], t0[kMaxGroup], t1[kMaxGroup];
  double c;
  for (int i = 0; i < n; ++i) {
    q0[i] = 0;
    q1[i] = half_group_2d_rows(probs[i].nao, probs[i].ncol, &c);
    t0[i] = q1[i];
    t1[i] = probs[i].nao;
  }
  hipError_t e = half_group_go<CfgQ128>(probs, n, s, q0, q1);
  if (e != hipSuccess) return e;
  return half_group_go<CfgH176>(probs, n, s, t0, t1);
}

hipError_t launch_half_group(const GroupHalf* probs, int n, int tile_n, hipStream_t s) {
  if (n < 1 || n > kMaxGroup) return hipErrorInvalidValue;
  switch (tile_n) {
    case 0:
    case 176: return half_group_go<CfgH176>(probs, n, s);
    case 96: return half_group_go<CfgH96>(probs, n, s);
    case 48: return half_group_go<CfgH48>(probs, n, s);
    case 128: return half_group_2d(probs, n, s);
    default: return hipErrorInvalidValue;
  }
}

template <class Cg>
static hipError_t syrk_group_go(const GroupSyrk* probs, int n, hipStream_t s) {
  SyrkGroup g{};
  g.n = n;
  g.start[0] = 0;
  bool clamp = false, flat_ok = true, flat_any = false;
  for (int p = 0; p < n; ++p) {
    const GroupSyrk& q = probs[p];
    SyrkDesc& d = g.d[p];
    d.A = q.A;
    d.n = q.n;
    d.nz = q.nz;
    const int64_t T = cdiv(q.n, Cg::BM);
    d.npairs = T * (T + 1) / 2;
    d.nsplit = q.nsplit;
    d.Kpart = q.Kpart;
    if (!offsets_fit(q.A) || q.nsplit < 1) return hipErrorInvalidValue;
    clamp = clamp || q.A.kc_n % 16 != 0;
    flat_ok = flat_ok && q.A.kc_n >= 16 && flat_fits(q.A);
    flat_any = flat_any || flat_pays(q.A);
    g.start[p + 1] = g.start[p] + d.npairs * d.nsplit * q.nz;
  }
  if (g.start[n] == 0) return hipSuccess;
  if (g.start[n] > 0x7fffffffLL) return hipErrorInvalidValue;
  // contraction chunks that are not whole slabs: one flat contraction per density (no padded
  // slabs) when every chunk is at least a slab long and the padding would cost
  const bool flat = clamp && flat_ok && flat_any;
  double cost[kMaxGroup];   // slabs of one split, plus about two for the prologue and the epilogue
  for (int p = 0; p < n; ++p) {
    const OpMap& A = g.d[p].A;
    cost[p] = (flat ? (double)cdiv(A.kb_n * A.kc_n, Cg::BK) / g.d[p].nsplit
                    : (double)cdiv(A.kb_n, g.d[p].nsplit) * (double)cdiv(A.kc_n, Cg::BK)) + 2.0;
  }
  const int64_t per = xcd_chunks(g.start, cost, n, g.xs);
  if (8 * per > 0x7fffffffLL) return hipErrorInvalidValue;
  if (flat) syrk_group_kernel<Cg, false, true><<<(unsigned)(8 * per), Cg::NT, 0, s>>>(g);
  else if (clamp) syrk_group_kernel<Cg, true><<<(unsigned)(8 * per), Cg::NT, 0, s>>>(g);
  else syrk_group_kernel<Cg, false><<<(unsigned)(8 * per), Cg::NT, 0, s>>>(g);
  return hipGetLastError();
}

int syrk_group_tile(const GroupSyrk* probs, int n) {
  int64_t nmax = 0;
  for (int p = 0; p < n; ++p) nmax = probs[p].n > nmax ? probs[p].n : nmax;
  return syrk_tile_for(nmax);
}

hipError_t launch_syrk_group(const GroupSyrk* probs, int n, int tile, hipStream_t s) {
  if (n < 1 || n > kMaxGroup) return hipErrorInvalidValue;
  if (tile == 0) tile = syrk_group_tile(probs, n);
  if (tile == CfgSyrk64::BM) return syrk_group_go<CfgSyrk64>(probs, n, s);
  if (tile == CfgSyrk::BM) return syrk_group_go<CfgSyrk>(probs, n, s);
  return hipErrorInvalidValue;
}

hipError_t launch_syrk_reduce(const double* Kpart, int nsplit, int64_t n, int64_t nz, double* K, hipStream_t s,
                              int accumulate) {
  const int64_t tot = n * n * nz;
  if (tot == 0) return hipSuccess;
  syrk_reduce_kernel<<<(unsigned)cdiv(tot, 256), 256, 0, s>>>(Kpart, nsplit, n, nz, K, accumulate);
  return hipGetLastError();
}

hipError_t launch_jvec(const double* X, int64_t naux, int64_t nao, int64_t ldx, const double* C, const double* w,
                       int64_t nocc, int64_t nz, double* v, hipStream_t s, int accumulate, int64_t ldv) {
  if (naux == 0 || nz == 0) return hipSuccess;
  if (nz > 65535 || naux > 0x7fffffffLL || (ldv != 0 && ldv < naux)) return hipErrorInvalidValue;
  jvec_kernel<<<dim3((unsigned)naux, (unsigned)nz), 256, 0, s>>>(X, nao, ldx, C, w, nocc, v, ldv ? ldv : naux,
                                                                  accumulate);
  return hipGetLastError();
}

hipError_t launch_coulomb(const double* B, int64_t naux, int64_t nao, const double* v, int64_t nz, double* J,
                          hipStream_t s, int accumulate, int64_t ldv) {
  const int64_t npair = nao * (nao + 1) / 2;
  if (ldv == 0) ldv = naux;
  if (ldv < naux) return hipErrorInvalidValue;
  for (int64_t z0 = 0; z0 < nz; z0 += kCoulombZ) {
    const int nzc = (int)(nz - z0 < kCoulombZ ? nz - z0 : kCoulombZ);
    coulomb_kernel<<<(unsigned)cdiv(npair, 256 * kCoulombPairs), 256, 0, s>>>(B, naux, nao, npair, v + z0 * ldv, nzc, ldv,
                                                               J + z0 * nao * nao, nao * nao, accumulate);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_add(const double* x, int64_t n, double* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  add_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(x, n, y);
  return hipGetLastError();
}

hipError_t launch_copy_rows(const double* x, int64_t rows, int64_t cols, double* y, int64_t ldy, int accumulate,
                            hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (ldy < cols) return hipErrorInvalidValue;
  copy_rows_kernel<<<(unsigned)cdiv(rows * cols, 256), 256, 0, s>>>(x, rows, cols, y, ldy, accumulate);
  return hipGetLastError();
}

hipError_t launch_scale_cols(const double* X, int64_t n, int64_t ncol, const double* w, double* Xw, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (ncol <= 0) return hipErrorInvalidValue;
  scale_cols_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(X, n, ncol, w, Xw);
  return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_zero_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(p, n);
  return hipGetLastError();
}

hipError_t launch_unpack_sym(const double* Jp, int64_t nz, int64_t nao, double* J, hipStream_t s) {
  const int64_t npair = nao * (nao + 1) / 2, tot = nz * npair;
  if (tot <= 0) return hipSuccess;
  unpack_sym_kernel<<<(unsigned)cdiv(tot, 256), 256, 0, s>>>(Jp, nz, nao, npair, J);
  return hipGetLastError();
}

hipError_t launch_chol_block(double* A, int64_t lda, int kb, double* Linv, int* info, int64_t k0, bool first,
                             hipStream_t s) {
  if (kb < 1 || kb > kCholNB) return hipErrorInvalidValue;
  chol_block_kernel<<<1, 256, 0, s>>>(A, lda, kb, Linv, info, k0, first ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_zero_upper(double* A, int64_t n, hipStream_t s) {
  if (n <= 1) return hipSuccess;
  zero_upper_kernel<<<(unsigned)cdiv(n * n, 256), 256, 0, s>>>(A, n);
  return hipGetLastError();
}

hipError_t launch_pack_lower(const double* A, int64_t nz, int64_t n, double* Ap, hipStream_t s) {
  const int64_t npair = n * (n + 1) / 2, tot = nz * npair;
  if (tot <= 0) return hipSuccess;
  pack_lower_kernel<<<(unsigned)cdiv(tot, 256), 256, 0, s>>>(A, nz, n, npair, Ap);
  return hipGetLastError();
}

hipError_t launch_fill_zero_strided(double* p, int64_t nz, int64_t s_z, int64_t n, hipStream_t s) {
  const int64_t tot = n * nz;
  if (tot <= 0) return hipSuccess;
  fill_zero_strided_kernel<<<(unsigned)cdiv(tot, 256), 256, 0, s>>>(p, nz, s_z, n);
  return hipGetLastError();
}

}  // namespace dfk
