// C-ABI entry points of libdfmi: argument checks, workspace planning, kernel orchestration.
#include "dfmi.h"
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <map>
#include <mutex>
#include <string>
#include <vector>

// Configuration of the grouped launches of df_batched_step: column tile of the half transform,
// K tile and the number of rounds of resident workgroups the K split counts aim at.
struct BatchedTune {
  int half_n, k_tile, k_rounds;
};

struct df_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  std::string err;
  // per-kernel timing (df_set_timing): events recorded on the context's stream
  struct Timed {
    int kind;
    hipEvent_t a, b;
  };
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<Timed> pending;
  hipEvent_t cur_a = nullptr;
  // autotuning of df_batched_step (df_set_autotune): configuration per problem-group shape,
  // keyed by "<gfx arch>|<shape>" (an empty arch: entries set by hand, valid on any device)
  bool autotune = false;
  std::map<std::string, BatchedTune> tune;
  std::string arch;          // the device's gfx name, looked up on the first tuning call
  bool arch_tried = false;
  std::string cache_path;    // DFMI_AUTOTUNE_CACHE at creation: loaded then, rewritten after tuning
  // split precision of the DF_PREC_SPLIT calls: slice count and the registered planes of B
  struct SplitReg {
    const double* B;
    int64_t naux, nao;
    const int8_t* Bs;
    const int* Be;
    int nslice;
  };
  int nslice = 7;
  std::vector<SplitReg> splits;
  // bound on the workspace of df_step_backward (0: none)
  size_t scratch_limit = 0;
};

namespace {

thread_local std::string g_create_err;

constexpr int64_t kMaxNao = 46340;   // keeps packed row offsets i(i+1)/2 + j inside 31 bits
constexpr size_t kAlign = 256;

df_status fail(df_ctx* c, df_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

std::string hip_msg(hipError_t e, const char* what) {
  return std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// A byte range of device memory the call reads or writes.
struct Range {
  const void* p;
  size_t bytes;
  const char* name;
  bool out;
};

// Inputs may share memory with each other; an output may overlap nothing else.
bool check_overlap(df_ctx* c, const std::vector<Range>& rs) {
  for (size_t a = 0; a < rs.size(); ++a)
    for (size_t b = a + 1; b < rs.size(); ++b) {
      if (!rs[a].out && !rs[b].out) continue;
      if (!rs[a].p || !rs[b].p || rs[a].bytes == 0 || rs[b].bytes == 0) continue;
      const char* x0 = (const char*)rs[a].p;
      const char* y0 = (const char*)rs[b].p;
      if (x0 < y0 + rs[b].bytes && y0 < x0 + rs[a].bytes) {
        c->err = std::string(rs[a].name) + " overlaps " + rs[b].name;
        return false;
      }
    }
  return true;
}

// Workspace carve-out, in the order the plan lists its pieces.
struct Plan {
  size_t total = 0;
  size_t take(int64_t ndoubles) {
    const size_t off = total;
    total += align_up((size_t)std::max<int64_t>(ndoubles, 0) * sizeof(double));
    return off;
  }
  // `bytes` at an offset that is a multiple of `align` (a power of two, at least kAlign)
  size_t take_bytes(int64_t bytes, size_t align) {
    total = (total + align - 1) / align * align;
    const size_t off = total;
    total += align_up((size_t)std::max<int64_t>(bytes, 0));
    return off;
  }
};

// Offsets of the workspace pieces of each operation.
struct StepPlan {
  size_t ccat, xo, xa, kpart, vtmp, vpart, bpu, buv;
  int nsplit;
};

// Workspace of df_ppaa.  The uv pairs run in chunks of `chunk`: W_uv [chunk][npair] and
// T_uv = W_uv Cq [chunk][nao][nq] are the per-chunk buffers, bounded by kPpaaChunkBytes.
constexpr int64_t kPpaaChunkBytes = int64_t(2) << 30;
struct PpaaPlan {
  size_t cpa, cpq, x, buv, vp, w, t;
  int64_t chunk;
};
PpaaPlan plan_ppaa(Plan& pl, int64_t naux, int64_t nao, int64_t nac, int64_t nq) {
  PpaaPlan p{};
  const int64_t npair = nao * (nao + 1) / 2, nuv = nac * (nac + 1) / 2;
  const int64_t per = (npair + nao * nq) * (int64_t)sizeof(double);
  p.chunk = std::max<int64_t>(1, std::min<int64_t>(nuv, kPpaaChunkBytes / std::max<int64_t>(per, 1)));
  p.cpa = pl.take(dfk::kpad16(nao) * nac);
  p.cpq = pl.take(dfk::kpad16(nao) * nq);
  p.x = pl.take(naux * nao * nac);
  p.buv = pl.take(naux * nac * nac);
  p.vp = pl.take(naux * nuv);
  p.w = pl.take(p.chunk * npair);
  p.t = pl.take(p.chunk * nao * nq);
  return p;
}

// Workspace of df_build_cholesky: the inverted diagonal blocks of L, a panel of the factorisation
// and one block row of the substitution.
struct BuildPlan {
  size_t linv, panel, t;
  int64_t nblk;
};
BuildPlan plan_build(Plan& pl, int64_t naux, int64_t nao) {
  BuildPlan p{};
  const int64_t nb = dfk::kCholNB, npair = nao * (nao + 1) / 2;
  p.nblk = (naux + nb - 1) / nb;
  p.linv = pl.take(p.nblk * nb * nb);
  p.panel = pl.take(naux * nb);
  p.t = pl.take(nb * npair);
  return p;
}

// Workspace of df_embed_cholesky: b^P M and M^T b^P M for a chunk of P (near 1 GiB).
constexpr int64_t kEmbedChunkBytes = int64_t(1) << 30;
struct EmbedPlan {
  size_t mpad, x, y;
  int64_t chunk;
};
EmbedPlan plan_embed(Plan& pl, int64_t naux, int64_t nao, int64_t nemb) {
  EmbedPlan p{};
  const int64_t per = (nao + nemb) * nemb * (int64_t)sizeof(double);
  p.chunk = std::max<int64_t>(1, std::min<int64_t>(naux, kEmbedChunkBytes / std::max<int64_t>(per, 1)));
  p.mpad = pl.take(dfk::kpad16(nao) * nemb);
  p.x = pl.take(p.chunk * nao * nemb);
  p.y = pl.take(p.chunk * nemb * nemb);
  return p;
}

// (pq|uv) of a batched problem: requested and not empty
bool wants_ppaa(const df_problem& q) { return q.ppaa && q.nac > 0 && q.np > 0; }
// One workspace region serves the (pq|uv) of every problem of a batch in turn: the largest.
size_t batched_ppaa_bytes(const df_problem* probs, int n) {
  size_t m = 0;
  for (int i = 0; i < n; ++i)
    if (wants_ppaa(probs[i])) {
      Plan pp;
      plan_ppaa(pp, probs[i].naux, probs[i].nao, probs[i].nac, probs[i].np);
      m = std::max(m, pp.total);
    }
  return m;
}

StepPlan plan_step(Plan& pl, int64_t naux, int64_t nao, int64_t nocc, int64_t nac, int64_t np, bool caller_x) {
  StepPlan p{};
  const int64_t ncol = nocc + nac;
  p.ccat = pl.take(dfk::kpad16(nao) * ncol);
  p.xo = pl.take(caller_x ? 0 : naux * nao * nocc);
  p.xa = pl.take(caller_x ? 0 : naux * nao * nac);
  p.nsplit = dfk::syrk_splits(nao, naux, 1);
  p.kpart = pl.take((int64_t)p.nsplit * nao * nao);
  p.vtmp = pl.take(naux);
  p.vpart = pl.take(nocc > 0 ? naux * dfk::half_tiles(nao, ncol) : 0);
  p.bpu = pl.take(naux * np * nac);
  p.buv = pl.take(naux * nac * nac);
  return p;
}

// Workspace of df_step_backward for chunks of `chunk` auxiliary rows.  flags: DF_BWD_GJ /
// DF_BWD_GK / DF_BWD_GERI say which cotangents are given, DF_CALLER_X that the forward's half
// transforms are passed in.  Per chunk: X_occ and X_act of its rows (when recomputed), Y_P = S X_P
// [P][kpad16(nao)][nocc], b_uv and Z; the split partials are sized for the most splits any chunk
// can take, so the total grows with the chunk.
struct BwdPlan {
  size_t ccat, xo, xa, g, u, upart, M, S, Y, kpart, Gs, buv, Z, apart;
  int64_t chunk;
};

BwdPlan plan_backward(Plan& pl, int64_t naux, int64_t nao, int64_t nocc, int64_t nac, int flags, int64_t chunk) {
  BwdPlan p{};
  const bool gj = flags & DF_BWD_GJ, gk = flags & DF_BWD_GK, ge = flags & DF_BWD_GERI;
  const bool cx = flags & DF_CALLER_X;
  const bool do_k = gk && nocc > 0, do_e = ge && nac > 0;
  const bool need_xo = do_k && !cx, need_xa = do_e && !cx;
  const int64_t npair = nao * (nao + 1) / 2, ch = chunk;
  p.chunk = chunk;
  p.ccat = pl.take(dfk::kpad16(nao) * ((need_xo ? nocc : 0) + (need_xa ? nac : 0)));
  p.xo = pl.take(need_xo ? ch * nao * nocc : 0);
  p.xa = pl.take(need_xa ? ch * nao * nac : 0);
  p.g = pl.take(gj && nocc > 0 ? npair : 0);
  p.u = pl.take(gj && nocc > 0 ? naux : 0);
  p.upart = pl.take(gj && nocc > 0 ? (int64_t)dfk::jvec_packed_chunks() * naux : 0);
  p.M = pl.take(gj && nocc > 0 ? nao * nao : 0);
  p.S = pl.take(do_k ? nao * nao : 0);
  p.Y = pl.take(do_k ? ch * dfk::kpad16(nao) * nocc : 0);
  p.kpart = pl.take(do_k ? dfk::half_reduce_part_bound(nao, nocc, ch) : 0);
  p.Gs = pl.take(do_e ? nac * nac * nac * nac : 0);
  p.buv = pl.take(do_e ? ch * nac * nac : 0);
  p.Z = pl.take(do_e ? ch * nac * nac : 0);
  p.apart = pl.take(do_e ? (int64_t)dfk::gemm_splits_bound(nao, nac, (ch * nac + 15) / 16) * nao * nac : 0);
  return p;
}

// Auxiliary rows per chunk of df_step_backward under a workspace bound: all of them without a
// bound, else the most whose workspace fits (the workspace grows with the chunk); 0 when not even
// one row fits.
int64_t backward_rows(int64_t naux, int64_t nao, int64_t nocc, int64_t nac, int flags, size_t limit) {
  if (limit == 0) return naux;
  auto need = [&](int64_t ch) {
    Plan pl;
    plan_backward(pl, naux, nao, nocc, nac, flags, ch);
    return pl.total;
  };
  if (need(1) > limit) return 0;
  int64_t lo = 1, hi = naux;   // need(lo) <= limit
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (need(mid) <= limit) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---- split precision ----
// Planes of an operand with `rows` rows and contraction length K (split_plane_bytes: 1 KB blocks
// of 32 rows x 32 k) and [rows] int32 exponents.  The planes start on a 4 KB boundary of the
// workspace: a block that straddles one (planes at 256 bytes past a 1 KB boundary) made the
// adjoint's slice product over (P, nu) 2-4 ms slower.
constexpr size_t kPlaneAlign = 4096;
struct SplitBuf {
  size_t planes, ex;
};
SplitBuf take_split(Plan& pl, int64_t rows, int64_t K, int nslice) {
  SplitBuf b{};
  const int64_t bytes = dfk::split_plane_bytes(rows, K, nslice);
  b.planes = pl.take_bytes(bytes, kPlaneAlign);
  b.ex = pl.take((rows * 4 + 7) / 8);
  return b;
}

// Split count for a slice product of `tiles` workgroup tiles and nks 32-deep steps: at least
// one workgroup per CU (one is resident per CU), at least 32 steps per split.  Long
// contractions are cut further, to at most kSliceSteps steps per split, so that the operand rows
// of the splits in flight stay within the 256 MB last-level cache; that is also below the
// longest split the int32 sums allow.
constexpr int64_t kSliceSteps = 512;
static_assert(kSliceSteps <= 1024, "a split longer than the exact int32 range");
int slice_splits(int64_t tiles, int64_t nks) {
  int64_t ns = tiles > 0 ? (256 + tiles - 1) / tiles : 1;
  const int64_t ns_cache = (nks + kSliceSteps - 1) / kSliceSteps;
  if (ns > nks / 32) ns = nks / 32;
  if (ns < ns_cache) ns = ns_cache;
  if (ns < 1) ns = 1;
  return (int)ns;
}

// ---- plans of the four calls that take DF_ACCUMULATE and DF_PREC_SPLIT ----
// Split-precision limits of these calls: every contraction (over nao, naux, or naux * nocc in
// K's splits) fits the int32-exact split length, and the plane rows stay below 2^31.
bool split_sizes_ok(int64_t naux, int64_t nao, int64_t rows) {
  return nao <= 32768 && naux <= 32768 && dfk::rpad32(naux * nao) <= 0x7fffffffLL && dfk::rpad32(rows) <= 0x7fffffffLL;
}

// df_half_transform.  FP64: the zero-padded C.  Split: planes of the rows c of C and, with C2, of
// the rows p of C2 and the rows (P, c) of X.  With DF_ACCUMULATE and C2, X of this call is
// formed in `xnew` (Y needs it alone) and then added to X.
struct HalfPlan {
  size_t cpad, xnew;
  SplitBuf cs, xs, c2s;
};
HalfPlan plan_half(Plan& pl, int64_t naux, int64_t nao, int64_t ncol, int64_t n2, int flags, int nslice) {
  HalfPlan p{};
  const bool acc = flags & DF_ACCUMULATE, sp = flags & DF_PREC_SPLIT;
  p.cpad = pl.take(sp ? 0 : dfk::kpad16(nao) * ncol);
  p.xnew = pl.take(acc && n2 > 0 ? naux * nao * ncol : 0);
  if (sp) {
    p.cs = take_split(pl, ncol, nao, nslice);
    p.xs = take_split(pl, n2 > 0 ? naux * ncol : 0, nao, nslice);
    p.c2s = take_split(pl, n2, nao, nslice);
  }
  return p;
}

// df_jk.  X = b^P [C_1 .. C_ndm] P-major [naux][nao][ndm*nocc]; v of this call in vtmp.  FP64: the
// padded operand, the K split partials.  Split: planes of the rows (z, c) of the factors, planes of
// every density's X_occ (rows m over (P, c)) and, with weights, of X diag(w) (xw) as the second
// operand of each K product.
struct JkPlan {
  size_t ccat, x, kpart, vtmp, xw;
  SplitBuf cs, xos, xws;
  int64_t xplane;   // bytes of the planes of one density's X_occ
  int nsplit;
};
// nsplit_fp64 > 0 sizes the FP64 K partials for that many splits instead of the call's own count.
JkPlan plan_jk(Plan& pl, int64_t naux, int64_t nao, int64_t ndm, int64_t nocc, bool weighted, int flags, int nslice,
               int nsplit_fp64 = 0) {
  JkPlan p{};
  const bool sp = flags & DF_PREC_SPLIT;
  const int64_t ncol = ndm * nocc;
  p.ccat = pl.take(sp ? 0 : dfk::kpad16(nao) * ncol);
  p.x = pl.take(naux * nao * ncol);
  p.vtmp = pl.take(ndm * naux);
  if (!sp) {
    p.nsplit = nsplit_fp64 > 0 ? nsplit_fp64 : dfk::syrk_splits(nao, naux, ndm);
  } else {
    p.cs = take_split(pl, ncol, nao, nslice);
    p.xplane = nocc > 0 ? dfk::split_plane_bytes(nao, naux * nocc, nslice) : 0;
    p.xos.planes = pl.take((ndm * p.xplane + 7) / 8);
    p.xos.ex = pl.take((ndm * nao * 4 + 7) / 8);
    p.xw = pl.take(weighted ? naux * nao * ncol : 0);
    p.xws.planes = pl.take(weighted ? (ndm * p.xplane + 7) / 8 : 0);
    p.xws.ex = pl.take(weighted ? (ndm * nao * 4 + 7) / 8 : 0);
    p.nsplit = nocc > 0 ? slice_splits(dfk::slice_gemm_tiles(nao, nao, true) * ndm,
                                       dfk::slice_gemm_steps(dfk::kpad64(naux * nocc)))
                        : 1;
  }
  p.kpart = pl.take((int64_t)p.nsplit * ndm * nao * nao);
  return p;
}

// ---- the static scratch of df_jk_noalloc ----
// df_jk_noalloc runs the JK call in blocks of auxiliary rows whose workspace fits this array, so it
// never allocates.  Host code must not pass `scratch` itself to a kernel (its name is a host-side
// stand-in there); it uses the address hipGetSymbolAddress returns on each device.
constexpr size_t kNoallocBytes = size_t(128) << 20;
static __device__ __align__(256) char scratch[kNoallocBytes];

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_addr;   // device -> address of `scratch` there

// K split count of df_jk_noalloc's blocks of r auxiliary rows: at most 4, so that the K partials
// leave room for X; non-decreasing in r.
int noalloc_jk_splits(int64_t nao, int64_t r, int64_t ndm) {
  return std::min(dfk::syrk_splits_bound(nao, r, ndm), 4);
}

// Auxiliary rows per block of df_jk_noalloc (FP64): the most whose workspace fits the scratch.  The
// workspace grows with the rows (the split count does not fall), so every block, the ragged last
// one too, fits; 0 when one row does not fit.
int64_t noalloc_jk_rows(int64_t naux, int64_t nao, int64_t ndm, int64_t nocc, bool weighted) {
  auto need = [&](int64_t r) {
    Plan pl;
    plan_jk(pl, r, nao, ndm, nocc, weighted, 0, 0, noalloc_jk_splits(nao, r, ndm));
    return pl.total;
  };
  if (need(1) > kNoallocBytes) return 0;
  int64_t lo = 1, hi = naux;   // need(lo) fits
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (need(mid) <= kNoallocBytes) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// df_active_eri: X_act AO-major [nao][naux][nac], b_uv of this call.  Split: planes of the rows u
// of Cact, of the rows (P, u) of X_act and of the rows uv of b_uv over P.
struct ActPlan {
  size_t cpad, x, buv;
  SplitBuf cas, xas, buvs;
};
ActPlan plan_act(Plan& pl, int64_t naux, int64_t nao, int64_t nac, int flags, int nslice) {
  ActPlan p{};
  const bool sp = flags & DF_PREC_SPLIT;
  p.cpad = pl.take(sp ? 0 : dfk::kpad16(nao) * nac);
  p.x = pl.take(naux * nao * nac);
  p.buv = pl.take(naux * nac * nac);
  if (sp) {
    p.cas = take_split(pl, nac, nao, nslice);
    p.xas = take_split(pl, naux * nac, nao, nslice);
    p.buvs = take_split(pl, nac * nac, naux, nslice);
  }
  return p;
}

// df_papa: X_act AO-major, b_pu and b_vw (default) or b_qv (DF_PAPA_FULL).  Split: planes of the
// rows of Cact, Cp (and Cq), of the rows (P, u) of X_act and of the rows of b_pu and b_vw / b_qv
// over P.
struct PapaPlan {
  size_t cpad, x, bpu, bvw, bqv;
  SplitBuf cas, cps, cqs, xas, bpus, bvws, bqvs;
};
PapaPlan plan_papa(Plan& pl, int64_t naux, int64_t nao, int64_t nac, int64_t np, int64_t nq, int flags, int nslice) {
  PapaPlan p{};
  const bool full = flags & DF_PAPA_FULL, sp = flags & DF_PREC_SPLIT;
  p.cpad = pl.take(sp ? 0 : dfk::kpad16(nao) * nac);
  p.x = pl.take(naux * nao * nac);
  p.bpu = pl.take(naux * np * nac);
  p.bvw = pl.take(full ? 0 : naux * nac * nac);
  p.bqv = pl.take(full ? naux * nq * nac : 0);
  if (sp) {
    p.xas = take_split(pl, naux * nac, nao, nslice);
    p.cps = take_split(pl, np, nao, nslice);
    p.bpus = take_split(pl, np * nac, naux, nslice);
    p.cas = take_split(pl, nac, nao, nslice);
    p.bvws = take_split(pl, full ? 0 : nac * nac, naux, nslice);
    p.cqs = take_split(pl, full ? nq : 0, nao, nslice);
    p.bqvs = take_split(pl, full ? nq * nac : 0, naux, nslice);
  }
  return p;
}

struct SplitMmPlan {
  SplitBuf a, b;
  size_t part;
  int nsplit;
};
SplitMmPlan plan_split_mm(Plan& pl, int64_t M, int64_t N, int64_t K, int nslice) {
  SplitMmPlan p{};
  p.a = take_split(pl, M, K, nslice);
  p.b = take_split(pl, N, K, nslice);
  p.nsplit = slice_splits(dfk::slice_gemm_tiles(M, N, false), dfk::slice_gemm_steps(dfk::kpad64(K)));
  p.part = pl.take(p.nsplit > 1 ? (int64_t)p.nsplit * M * N : 0);
  return p;
}

// Workspace of df_step_split (forward in split precision; B comes pre-split).
struct StepSplitPlan {
  size_t ccat, xo, xa, bpu, buv, kpart, vtmp;
  SplitBuf cs, xos, xas, cps, cas, bpus, buvs;
  int nsk;
};
StepSplitPlan plan_step_split(Plan& pl, int64_t naux, int64_t nao, int64_t nocc, int64_t nac, int64_t np,
                              int nslice, bool caller_x) {
  StepSplitPlan p{};
  const int64_t ncol = nocc + nac;
  p.ccat = pl.take(nao * ncol);
  p.xo = pl.take(caller_x ? 0 : naux * nao * nocc);   // P-major [naux][nao][nocc]
  p.xa = pl.take(caller_x ? 0 : naux * nao * nac);    // AO-major [nao][naux][nac]
  p.bpu = pl.take(naux * np * nac);
  p.buv = pl.take(naux * nac * nac);
  p.cs = take_split(pl, ncol, nao, nslice);
  p.xos = take_split(pl, nocc > 0 ? nao : 0, naux * nocc, nslice);
  p.nsk = slice_splits(dfk::slice_gemm_tiles(nao, nao, true), dfk::slice_gemm_steps(dfk::kpad64(naux * nocc)));
  p.kpart = pl.take(nocc > 0 ? (int64_t)p.nsk * nao * nao : 0);
  p.vtmp = pl.take(naux);
  p.xas = take_split(pl, naux * nac, nao, nslice);
  p.cps = take_split(pl, nac > 0 ? np : 0, nao, nslice);
  p.cas = take_split(pl, nac, nao, nslice);
  p.bpus = take_split(pl, np * nac, naux, nslice);
  p.buvs = take_split(pl, nac * nac, naux, nslice);
  return p;
}

// Workspace of df_step_backward_split: the Coulomb and active parts as in df_step_backward
// (FP64), the exchange part as slice products.
struct BwdSplitPlan {
  BwdPlan f;
  size_t S, Y, part;
  SplitBuf ys;
  int nsk;
};
BwdSplitPlan plan_backward_split(Plan& pl, int64_t naux, int64_t nao, int64_t nocc, int64_t nac, int flags,
                                 int nslice) {
  BwdSplitPlan p{};
  p.f = plan_backward(pl, naux, nao, nocc, nac, (flags & ~DF_BWD_GK) | DF_CALLER_X, naux);
  p.nsk = 1;
  if ((flags & DF_BWD_GK) && nocc > 0) {
    p.S = pl.take(nao * nao);
    p.Y = pl.take(naux * nao * nocc);   // P-major [naux][nao][nocc]
    p.ys = take_split(pl, nocc, naux * nao, nslice);
    p.nsk = slice_splits(dfk::slice_gemm_tiles(nao, nocc, false), dfk::slice_gemm_steps(dfk::kpad64(naux * nao)));
    p.part = pl.take(p.nsk > 1 ? (int64_t)p.nsk * nao * nocc : 0);
  }
  return p;
}

// ---- batched problems ----
struct BatchedPiece {
  size_t cpad, xo, xa, v, jp, kpart, buv, bpu, dfull, dw, vpart;
  int nsplit, vsplit;
};
int64_t batched_ncol(const df_problem& q) { return q.ndm * q.nocc + q.nac; }
// half-transform work of a problem, for the largest-first order
int64_t batched_work(const df_problem& q) { return q.naux * q.nao * q.nao * batched_ncol(q); }

// Split counts of the grouped K launch: every (density, split, tile pair) item gets about the
// same number of 16-deep slabs, about sixteen rounds of resident workgroups in all, so that
// the long contractions of the big problems do not run alone at the end.
// Candidate configurations the autotuner times (the first of each is the default).
constexpr int kHalfTiles[] = {176, 96, 48, 128};
constexpr int kKTiles[] = {64, 128};
constexpr int kKRounds[] = {16, 4, 64};

int batched_default_k_tile(const df_problem* probs, int n) {
  int64_t nmax = 0;
  for (int i = 0; i < n; ++i)
    if (probs[i].K && probs[i].nocc > 0) nmax = std::max(nmax, probs[i].nao);
  return dfk::syrk_tile_for(nmax);
}

// Split counts of the grouped K launch for K tile T: every (density, split, tile pair) item gets
// about the same number of 16-deep slabs, about `rounds` rounds of resident workgroups in all, so
// that the long contractions of the big problems do not run alone at the end.
std::vector<int> batched_k_splits(const df_problem* probs, int n, int T, int rounds) {
  double total = 0.0;
  for (int i = 0; i < n; ++i) {
    const df_problem& q = probs[i];
    if (!q.K || q.nocc <= 0) continue;
    const int64_t t = (q.nao + T - 1) / T;
    total += (double)(t * (t + 1) / 2) * q.ndm * q.naux * ((q.nocc + 15) / 16);
  }
  const double target = std::max(64.0, total / (rounds * 512.0));   // slabs per item
  std::vector<int> ns((size_t)n, 1);
  for (int i = 0; i < n; ++i) {
    const df_problem& q = probs[i];
    if (!q.K || q.nocc <= 0) continue;
    const double slabs = (double)q.naux * ((q.nocc + 15) / 16);
    ns[(size_t)i] = (int)std::min<double>((double)q.naux, std::max(1.0, std::ceil(slabs / target)));
  }
  return ns;
}

// The most splits any candidate configuration asks for (the workspace holds that many partials).
std::vector<int> batched_k_splits_max(const df_problem* probs, int n) {
  std::vector<int> m((size_t)n, 1);
  for (int T : kKTiles)
    for (int r : kKRounds) {
      const std::vector<int> ns = batched_k_splits(probs, n, T, r);
      for (int i = 0; i < n; ++i) m[(size_t)i] = std::max(m[(size_t)i], ns[(size_t)i]);
    }
  return m;
}

// The half-transform tile by the padded-area estimate: 2-D tiles (128) or one row of waves (176).
int batched_default_half_tile(const df_problem* probs, int n) {
  std::vector<int64_t> nao, ncol;
  for (int i = 0; i < n; ++i) {
    nao.push_back(probs[i].nao);
    ncol.push_back(batched_ncol(probs[i]));
  }
  return n > 0 ? dfk::half_group_tile_for(nao.data(), ncol.data(), n) : kHalfTiles[0];
}

BatchedTune batched_default_tune(const df_problem* probs, int n) {
  return BatchedTune{batched_default_half_tile(probs, n), batched_default_k_tile(probs, n), kKRounds[0]};
}

// The shape of a problem group: what the work and hence the best configuration depend on.
std::string batched_key(const df_problem* probs, int n) {
  std::string k;
  for (int i = 0; i < n; ++i) {
    const df_problem& q = probs[i];
    char buf[160];
    std::snprintf(buf, sizeof buf, "%lld,%lld,%lld,%lld,%lld,%lld,%d%d%d%d;", (long long)q.naux, (long long)q.nao,
                  (long long)q.ndm, (long long)q.nocc, (long long)q.nac, (long long)q.np, q.J != nullptr,
                  q.K != nullptr, q.eri != nullptr, q.papa != nullptr);
    k += buf;
  }
  return k;
}

// ---- the autotuning table and its file ----
// The device's gfx name ("gfx950"), asked of the runtime once; empty where there is no device.
void resolve_arch(df_ctx* c) {
  if (!c->arch.empty() || c->arch_tried) return;
  c->arch_tried = true;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  const std::string name(prop.gcnArchName);
  c->arch = name.substr(0, name.find(':'));
}

// An entry's key is "<arch>|<shape>": choices measured on a device carry its gfx name, choices set
// by hand (df_batched_set_tuning) carry none and hold on any device.
const BatchedTune* tune_find(const df_ctx* c, const std::string& shape) {
  if (!c->arch.empty()) {
    const auto it = c->tune.find(c->arch + "|" + shape);
    if (it != c->tune.end()) return &it->second;
  }
  const auto it = c->tune.find("|" + shape);
  return it != c->tune.end() ? &it->second : nullptr;
}

bool tune_valid(const BatchedTune& t) {
  auto in = [](int v, const int* set, int n) { return std::find(set, set + n, v) != set + n; };
  return in(t.half_n, kHalfTiles, 4) && in(t.k_tile, kKTiles, 2) && in(t.k_rounds, kKRounds, 3);
}

// The value of "name" in one flat JSON object (a string without escapes, or an integer).
bool json_field(const std::string& obj, const char* name, std::string* str, long long* num) {
  const std::string pat = std::string("\"") + name + "\"";
  size_t p = obj.find(pat);
  if (p == std::string::npos) return false;
  p = obj.find(':', p + pat.size());
  if (p == std::string::npos) return false;
  ++p;
  while (p < obj.size() && (obj[p] == ' ' || obj[p] == '\t' || obj[p] == '\n' || obj[p] == '\r')) ++p;
  if (p >= obj.size()) return false;
  if (obj[p] == '"') {
    const size_t q = obj.find('"', p + 1);
    if (q == std::string::npos || !str) return false;
    *str = obj.substr(p + 1, q - p - 1);
    return true;
  }
  if (!num) return false;
  char* end = nullptr;
  *num = std::strtoll(obj.c_str() + p, &end, 10);
  return end != obj.c_str() + p;
}

// Entries of a tuning file (format dfmi-autotune/1) merged into the table; entries of other
// operations, precisions or unknown configurations are skipped.  A missing file is an error.
bool tune_read(df_ctx* c, const std::string& path, std::string* err) {
  std::ifstream f(path);
  if (!f) {
    *err = "cannot open " + path;
    return false;
  }
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  if (text.find("\"dfmi-autotune/1\"") == std::string::npos) {
    *err = path + " is not a dfmi-autotune/1 file";
    return false;
  }
  const size_t list = text.find("\"entries\"");
  for (size_t p = list == std::string::npos ? text.size() : text.find('{', list); p < text.size();
       p = text.find('{', p + 1)) {
    const size_t q = text.find('}', p);
    if (q == std::string::npos) break;
    const std::string obj = text.substr(p, q - p + 1);
    std::string op, prec, arch, shape;
    long long h = 0, kt = 0, kr = 0;
    if (json_field(obj, "op", &op, nullptr) && op == "df_batched_step" && json_field(obj, "precision", &prec, nullptr) &&
        prec == "fp64" && json_field(obj, "arch", &arch, nullptr) && json_field(obj, "shape", &shape, nullptr) &&
        json_field(obj, "half_tile_n", nullptr, &h) && json_field(obj, "k_tile", nullptr, &kt) &&
        json_field(obj, "k_rounds", nullptr, &kr)) {
      const BatchedTune t{(int)h, (int)kt, (int)kr};
      if (tune_valid(t)) c->tune[arch + "|" + shape] = t;
    }
    p = q;
  }
  return true;
}

// The whole table as a tuning file, written to a temporary name and renamed into place.
bool tune_write(const df_ctx* c, const std::string& path, std::string* err) {
  const std::string tmp = path + ".tmp" + std::to_string((unsigned long long)(uintptr_t)c);
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) {
      *err = "cannot write " + tmp;
      return false;
    }
    f << "{\n  \"format\": \"dfmi-autotune/1\",\n  \"entries\": [";
    bool first = true;
    for (const auto& e : c->tune) {
      const size_t bar = e.first.find('|');
      f << (first ? "\n" : ",\n") << "    {\"op\": \"df_batched_step\", \"precision\": \"fp64\", \"arch\": \""
        << e.first.substr(0, bar) << "\", \"shape\": \"" << e.first.substr(bar + 1) << "\", \"half_tile_n\": "
        << e.second.half_n << ", \"k_tile\": " << e.second.k_tile << ", \"k_rounds\": " << e.second.k_rounds << "}";
      first = false;
    }
    f << "\n  ]\n}\n";
    if (!f) {
      *err = "error writing " + tmp;
      return false;
    }
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) {
    std::remove(tmp.c_str());
    *err = "cannot rename " + tmp + " to " + path;
    return false;
  }
  return true;
}

// J of many densities as one product: Jp[z][pair] = sum_P v[z][P] b^P[pair] (then unpacked)
bool batched_j_gemm(const df_problem& q) { return q.ndm > 4; }

// The J-vectors from packed B and the packed densities (v = Dw B^T) instead of from X_occ, when
// X_occ (naux nao ndm nocc) is the larger of the two to read (B: naux npair).
bool batched_jvec_from_b(const df_problem& q) { return q.J && q.nocc > 0 && 2 * q.ndm * q.nocc > q.nao + 1; }

std::vector<BatchedPiece> plan_batched(Plan& pl, const df_problem* probs, int n) {
  std::vector<BatchedPiece> v((size_t)n);
  const std::vector<int> ks = batched_k_splits_max(probs, n);
  for (int i = 0; i < n; ++i) {
    const df_problem& q = probs[i];
    BatchedPiece& b = v[(size_t)i];
    const int64_t ncol = batched_ncol(q);
    const bool need_x = ncol > 0 && (q.J || q.K || q.eri || q.papa);
    b.cpad = pl.take(need_x ? dfk::kpad16(q.nao) * ncol : 0);
    b.xo = pl.take(need_x ? q.naux * q.nao * q.ndm * q.nocc : 0);   // P-major [naux][nao][ndm*nocc]
    b.xa = pl.take(need_x ? q.naux * q.nao * q.nac : 0);            // AO-major [nao][naux][nac]
    b.v = pl.take(q.J && q.nocc > 0 ? q.ndm * q.naux : 0);
    const int64_t npair = q.nao * (q.nao + 1) / 2;
    b.dfull = pl.take(batched_jvec_from_b(q) ? q.ndm * q.nao * q.nao : 0);
    b.dw = pl.take(batched_jvec_from_b(q) ? q.ndm * npair : 0);
    b.vsplit = batched_jvec_from_b(q) ? dfk::gemm_splits(q.ndm, q.naux, (npair + 15) / 16) : 1;
    b.vpart = pl.take(b.vsplit > 1 ? (int64_t)b.vsplit * q.ndm * q.naux : 0);
    b.jp = pl.take(q.J && q.nocc > 0 && batched_j_gemm(q) ? q.ndm * q.nao * (q.nao + 1) / 2 : 0);
    b.nsplit = ks[(size_t)i];
    b.kpart = pl.take(q.K && q.nocc > 0 ? (int64_t)b.nsplit * q.ndm * q.nao * q.nao : 0);
    b.buv = pl.take(q.eri && q.nac > 0 ? q.naux * q.nac * q.nac : 0);
    b.bpu = pl.take(q.papa && q.nac > 0 && q.np > 0 ? q.naux * q.np * q.nac : 0);
  }
  return v;
}

// Workspace of one problem of df_batched_step_split (problems run one after another and share
// one region, sized for the largest).
struct SplitPiece {
  size_t cc, xo, xa, v, jp, dfull, dw, vpart, kpart, buv, bpu;
  SplitBuf cs, xos, xas, cas, cps, buvs, bpus;
  int64_t xplane;   // bytes of the planes of one density's X_occ
  int vsplit, nsk;
};
SplitPiece plan_split_piece(Plan& pl, const df_problem& q, int nslice, bool k_fp64) {
  SplitPiece b{};
  const int64_t ncol = batched_ncol(q), no = q.ndm * q.nocc, npair = q.nao * (q.nao + 1) / 2;
  const bool need_x = ncol > 0 && (q.J || q.K || q.eri || q.papa);
  const bool dj = q.J && q.nocc > 0, dk = q.K && q.nocc > 0;
  const bool de = q.eri && q.nac > 0, dp = q.papa && q.nac > 0 && q.np > 0;
  b.cc = pl.take(need_x ? q.nao * ncol : 0);
  b.cs = take_split(pl, need_x ? ncol : 0, q.nao, nslice);
  b.xo = pl.take(need_x ? q.naux * q.nao * no : 0);          // P-major [naux][nao][ndm*nocc]
  b.xa = pl.take(need_x ? q.naux * q.nao * q.nac : 0);      // AO-major [nao][naux][nac]
  b.v = pl.take(dj ? q.ndm * q.naux : 0);
  b.jp = pl.take(dj && batched_j_gemm(q) ? q.ndm * npair : 0);
  b.dfull = pl.take(batched_jvec_from_b(q) ? q.ndm * q.nao * q.nao : 0);
  b.dw = pl.take(batched_jvec_from_b(q) ? q.ndm * npair : 0);
  b.vsplit = batched_jvec_from_b(q) ? dfk::gemm_splits(q.ndm, q.naux, (npair + 15) / 16) : 1;
  b.vpart = pl.take(b.vsplit > 1 ? (int64_t)b.vsplit * q.ndm * q.naux : 0);
  const bool dks = dk && !k_fp64;   // K from int8 slices of every density's X_occ
  b.xplane = dks ? dfk::split_plane_bytes(q.nao, q.naux * q.nocc, nslice) : 0;
  b.xos.planes = pl.take((q.ndm * b.xplane + 7) / 8);
  b.xos.ex = pl.take(dks ? (q.ndm * q.nao * 4 + 7) / 8 : 0);
  b.nsk = !dk ? 1
          : dks ? slice_splits(dfk::slice_gemm_tiles(q.nao, q.nao, true) * q.ndm,
                               dfk::slice_gemm_steps(dfk::kpad64(q.naux * q.nocc)))
                : dfk::syrk_splits(q.nao, q.naux, q.ndm);
  b.kpart = pl.take(dk ? (int64_t)b.nsk * q.ndm * q.nao * q.nao : 0);
  b.xas = take_split(pl, de || dp ? q.naux * q.nac : 0, q.nao, nslice);
  b.cas = take_split(pl, de ? q.nac : 0, q.nao, nslice);
  b.buv = pl.take(de ? q.naux * q.nac * q.nac : 0);
  b.buvs = take_split(pl, de ? q.nac * q.nac : 0, q.naux, nslice);
  b.cps = take_split(pl, dp ? q.np : 0, q.nao, nslice);
  b.bpu = pl.take(dp ? q.naux * q.np * q.nac : 0);
  b.bpus = take_split(pl, dp ? q.np * q.nac : 0, q.naux, nslice);
  return b;
}

df_status check_ctx(df_ctx* c) {
  if (!c) return DF_ERR_ARG;
  c->err.clear();
  return DF_OK;
}

df_status check_core(df_ctx* c, const double* B, int64_t naux, int64_t nao) {
  if (!B) return fail(c, DF_ERR_ARG, "B is NULL");
  if (naux < 1 || nao < 1) return fail(c, DF_ERR_SHAPE, "naux and nao must be >= 1");
  if (nao > kMaxNao) return fail(c, DF_ERR_SHAPE, "nao exceeds 46340");
  return DF_OK;
}

df_status need_ws(df_ctx* c, size_t bytes) {
  if (bytes == 0) return DF_OK;
  if (!c->ws) return fail(c, DF_ERR_WORKSPACE, "no workspace attached (need " + std::to_string(bytes) + " bytes)");
  if (c->ws_bytes < bytes)
    return fail(c, DF_ERR_WORKSPACE, "workspace has " + std::to_string(c->ws_bytes) + " bytes, need " +
                                          std::to_string(bytes));
  return DF_OK;
}

df_status enter(df_ctx* c) {
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return fail(c, DF_ERR_HIP, hip_msg(e, "hipSetDevice"));
  return DF_OK;
}

#define DF_HIP(call, what)                                             \
  do {                                                                 \
    hipError_t e_ = (call);                                            \
    if (e_ != hipSuccess) return fail(c, DF_ERR_HIP, hip_msg(e_, what)); \
  } while (0)

df_status take_event(df_ctx* c, hipEvent_t* ev) {
  if (!c->ev_pool.empty()) {
    *ev = c->ev_pool.back();
    c->ev_pool.pop_back();
    return DF_OK;
  }
  DF_HIP(hipEventCreate(ev), "hipEventCreate");
  return DF_OK;
}

df_status timing_begin(df_ctx* c) {
  if (!c->timing) return DF_OK;
  if (df_status s = take_event(c, &c->cur_a)) return s;
  DF_HIP(hipEventRecord(c->cur_a, c->stream), "hipEventRecord");
  return DF_OK;
}

df_status timing_end(df_ctx* c, int kind) {
  if (!c->timing) return DF_OK;
  hipEvent_t b;
  if (df_status s = take_event(c, &b)) return s;
  DF_HIP(hipEventRecord(b, c->stream), "hipEventRecord");
  c->pending.push_back({kind, c->cur_a, b});
  return DF_OK;
}

// A kernel launch, bracketed by timing events when timing is on.
#define DF_LAUNCH(kind, call, what)                                      \
  do {                                                                   \
    if (df_status s_ = timing_begin(c)) return s_;                      \
    hipError_t e_ = (call);                                              \
    if (e_ != hipSuccess) return fail(c, DF_ERR_HIP, hip_msg(e_, what)); \
    if (df_status s_ = timing_end(c, kind)) return s_;                  \
  } while (0)

size_t dbytes(int64_t n) { return (size_t)std::max<int64_t>(n, 0) * sizeof(double); }

// ---- building blocks on the device ----

// T_P = b^P C (ncol columns of C, row stride ldc), written through `out` with z = P
// A block of columns of the dense half-transform operand: src [nao][ncols] (row stride ld) goes to
// columns [col0, col0 + ncols).
struct ColBlock {
  const double* src;
  int64_t ld, ncols, col0;
};

// cpad [kpad16(nao)][ncol] = the blocks side by side, rows nao.. zero.
df_status pad_operand(df_ctx* c, double* cpad, int64_t nao, int64_t ncol, const ColBlock* blocks, int nb) {
  for (int i = 0; i < nb; ++i) {
    const ColBlock& b = blocks[i];
    if (b.ncols == 0) continue;
    DF_LAUNCH(DF_KERNEL_OTHER,
              hipMemcpy2DAsync(cpad + b.col0, ncol * sizeof(double), b.src, b.ld * sizeof(double),
                               b.ncols * sizeof(double), nao, hipMemcpyDeviceToDevice, c->stream),
              "operand gather");
  }
  const int64_t kp = dfk::kpad16(nao);
  if (kp > nao)
    DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(cpad + nao * ncol, (kp - nao) * ncol, c->stream), "fill");
  return DF_OK;
}

// cc [nao][ncol] = the blocks side by side (no padding)
df_status pad_operand_plain(df_ctx* c, double* cc, int64_t nao, int64_t ncol, const ColBlock* blocks, int nb) {
  for (int i = 0; i < nb; ++i) {
    const ColBlock& b = blocks[i];
    if (b.ncols == 0) continue;
    DF_LAUNCH(DF_KERNEL_OTHER,
              hipMemcpy2DAsync(cc + b.col0, ncol * sizeof(double), b.src, b.ld * sizeof(double),
                               b.ncols * sizeof(double), nao, hipMemcpyDeviceToDevice, c->stream),
              "operand gather");
  }
  return DF_OK;
}

// half transform against a padded operand from pad_operand
df_status run_half(df_ctx* c, const double* B, int64_t naux, int64_t nao, const double* cpad, int64_t ncol,
                   const dfk::OutMap& out) {
  DF_LAUNCH(DF_KERNEL_HALF_TRANSFORM, dfk::launch_half_transform(B, naux, nao, cpad, ncol, ncol, out, c->stream),
            "half transform launch");
  return DF_OK;
}

// X P-major [naux][nao][ld] (all ncol columns)
dfk::OutMap out_pmajor(double* X, int64_t naux, int64_t nao, int64_t ncol, int64_t ld) {
  (void)naux;
  dfk::OutMap o = dfk::out_plain(X, nao, ncol, ld);
  o.s_z = nao * ld;
  return o;
}

// columns [0, nocc) to Xo P-major [naux][nao][nocc], columns [nocc, nocc+nac) to Xa AO-major [nao][naux][nac]
dfk::OutMap out_split(double* Xo, double* Xa, int64_t naux, int64_t nao, int64_t nocc, int64_t nac) {
  dfk::OutMap o = dfk::out_plain(Xo, nao, nocc + nac, nocc);
  o.s_z = nao * nocc;
  o.nsplit = nocc;
  o.p2 = Xa;
  o.s2_m = naux * nac;
  o.s2_z = nac;
  return o;
}

// out[P][p][u] = sum_mu Cl[mu][p] Xa[mu][P][u]  (Cl is [nao][nl], Xa AO-major: rows mu of stride ld,
// columns (P, u) for P < naux)
df_status run_mo_ld(df_ctx* c, const double* Cl, int64_t nl, const double* Xa, int64_t ld, int64_t naux, int64_t nao,
                    int64_t nr, double* out) {
  if (nl == 0 || nr == 0) return DF_OK;
  const int kind = DF_KERNEL_MO_TRANSFORM;
  const dfk::OpMap A = dfk::op_map(Cl, nl, 1, nao, nl);
  const dfk::OpMap Bm = dfk::op_map(Xa, naux * nr, 1, nao, ld);
  dfk::OutMap O = dfk::out_plain(out, nl, naux * nr, nr);
  O.nl = nr;
  O.s_nh = nl * nr;
  DF_LAUNCH(kind, dfk::launch_gemm(A, Bm, O, 1, c->stream), "second transform launch");
  return DF_OK;
}

// run_mo_ld for Xa AO-major [nao][naux][nr]
df_status run_mo(df_ctx* c, const double* Cl, int64_t nl, const double* Xa, int64_t naux, int64_t nao, int64_t nr,
                 double* out) {
  return run_mo_ld(c, Cl, nl, Xa, naux * nr, naux, nao, nr, out);
}

// Y[P][p][c] (+)= sum_mu C2[mu][p] X[P][mu][c]  (X P-major [naux][nao][ncol]), batched over P
df_status run_mo_pmajor(df_ctx* c, const double* C2, int64_t n2, const double* X, int64_t naux, int64_t nao,
                        int64_t ncol, double* Y, int accumulate = 0) {
  if (n2 == 0 || ncol == 0) return DF_OK;
  const dfk::OpMap A = dfk::op_map(C2, n2, 1, nao, n2);
  dfk::OpMap Bm = dfk::op_map(X, ncol, 1, nao, ncol);
  Bm.s_z = nao * ncol;
  dfk::OutMap O = dfk::out_plain(Y, n2, ncol, ncol);
  O.s_z = n2 * ncol;
  O.accumulate = accumulate;
  for (int64_t p0 = 0; p0 < naux; p0 += 65535) {
    const int64_t np_ = std::min<int64_t>(65535, naux - p0);
    dfk::OpMap Bp = Bm;
    Bp.p = X + p0 * nao * ncol;
    dfk::OutMap Op = O;
    Op.p = Y + p0 * n2 * ncol;
    DF_LAUNCH(DF_KERNEL_MO_TRANSFORM, dfk::launch_gemm(A, Bp, Op, np_, c->stream), "second transform launch");
  }
  return DF_OK;
}

// out[m][n] (+)= sum_P L[P][m] R[P][n]
df_status run_pgemm(df_ctx* c, int kind, const double* L, int64_t M, const double* R, int64_t N, int64_t naux,
                    double* out, int accumulate = 0) {
  if (M == 0 || N == 0) return DF_OK;
  const dfk::OpMap A = dfk::op_map(L, M, 1, naux, M);
  const dfk::OpMap Bm = dfk::op_map(R, N, 1, naux, N);
  dfk::OutMap O = dfk::out_plain(out, M, N, N);
  O.accumulate = accumulate;
  DF_LAUNCH(kind, dfk::launch_gemm(A, Bm, O, 1, c->stream), "aux contraction launch");
  return DF_OK;
}

// K[z] (+)= sum_P X_z[P] diag(w_z) X_z[P]^T with X_z[P][i][c] = X[P][i][z*nocc + c]  (w may be NULL)
df_status run_k(df_ctx* c, const double* X, const double* w, int64_t naux, int64_t nao, int64_t ldx,
                int64_t nocc, int64_t nz, int nsplit, double* kpart, double* K, int accumulate = 0) {
  dfk::OpMap A = dfk::op_map(X, nao, ldx, nocc, 1);
  A.kb_n = naux;
  A.s_kb = nao * ldx;
  A.s_z = nocc;
  dfk::OpMap Bw = A;
  Bw.ks = w;
  Bw.s_ksz = nocc;
  DF_LAUNCH(DF_KERNEL_K_SYRK, dfk::launch_syrk_partial(A, Bw, nao, nz, nsplit, kpart, c->stream), "K tiles launch");
  DF_LAUNCH(DF_KERNEL_K_REDUCE, dfk::launch_syrk_reduce(kpart, nsplit, nao, nz, K, c->stream, accumulate),
            "K reduce launch");
  return DF_OK;
}

// ---- split-precision building blocks ----
// Planes and exponents of a split operand in the workspace.
struct SplitOp {
  int8_t* planes;
  int* ex;
};
SplitOp split_in(char* ws, const SplitBuf& b) { return SplitOp{(int8_t*)(ws + b.planes), (int*)(ws + b.ex)}; }

// the rows of operand o (contraction length K) cut into int8 planes
df_status split_of(df_ctx* c, const dfk::OpMap& o, int64_t K, int nslice, SplitOp d) {
  DF_LAUNCH(DF_KERNEL_SPLIT, dfk::launch_split_rows(o, K, nslice, d.planes, d.ex, c->stream), "split launch");
  return DF_OK;
}

// O(m, n) = sum_k a(m, k) b(n, k) from the planes of the M rows of a and the N rows of b (K <= 32768)
df_status slice_product(df_ctx* c, int kind, SplitOp a, int64_t M, SplitOp b, int64_t N, int64_t K, int nslice,
                        const dfk::OutMap& O) {
  DF_LAUNCH(kind,
            dfk::launch_slice_gemm(a.planes, a.ex, M, b.planes, b.ex, N, dfk::kpad64(K), nslice, O, false, 1, nullptr,
                                   c->stream),
            "slice product launch");
  return DF_OK;
}

// Rows (P, mu) of b^P times C over nu (Eq. ao2mo_1) from the registered planes of B and the planes
// of the ncol rows of C, written through OX (rows P * nao + mu, columns c).
df_status split_half(df_ctx* c, const df_ctx::SplitReg& r, SplitOp cs, int64_t ncol, const dfk::OutMap& OX) {
  DF_LAUNCH(DF_KERNEL_HALF_TRANSFORM,
            dfk::launch_slice_gemm(r.Bs, r.Be, r.naux * r.nao, cs.planes, cs.ex, ncol, dfk::kpad64(r.nao), r.nslice, OX,
                                   false, 1, nullptr, c->stream),
            "slice product launch");
  return DF_OK;
}

// The registered split of B for the context's slice count, or NULL.
const df_ctx::SplitReg* find_split(const df_ctx* c, const double* B, int64_t naux, int64_t nao) {
  for (const auto& r : c->splits)
    if (r.B == B && r.naux == naux && r.nao == nao && r.nslice == c->nslice) return &r;
  return nullptr;
}

// The split of B a DF_PREC_SPLIT call uses, with its planes appended to the call's input ranges.
df_status split_for_call(df_ctx* c, const double* B, int64_t naux, int64_t nao, int64_t rows,
                         const df_ctx::SplitReg** reg, std::vector<Range>& rs) {
  *reg = find_split(c, B, naux, nao);
  if (!*reg)
    return fail(c, DF_ERR_ARG, "DF_PREC_SPLIT: no split of B with " + std::to_string(c->nslice) +
                                   " slices is registered on this context (df_register_split)");
  if (!split_sizes_ok(naux, nao, rows))
    return fail(c, DF_ERR_SHAPE, "problem too large for the split path (nao, naux <= 32768, rows < 2^31)");
  rs.push_back({(*reg)->Bs, (size_t)dfk::split_plane_bytes(naux * nao, nao, (*reg)->nslice), "Bs", false});
  rs.push_back({(*reg)->Be, (size_t)naux * nao * 4, "Be", false});
  return DF_OK;
}

}  // namespace

extern "C" {

df_status df_create(df_ctx** ctx, int device, void* stream) {
  // No HIP call here: the device is selected (and checked) by the first call that
  // enqueues work, so a context can be created and its argument checks exercised
  // on a machine without a GPU.
  g_create_err.clear();
  if (!ctx) {
    g_create_err = "ctx is NULL";
    return DF_ERR_ARG;
  }
  *ctx = nullptr;
  if (device < 0) {
    g_create_err = "device must be >= 0";
    return DF_ERR_ARG;
  }
  df_ctx* c = new df_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  // a tuning file named by DFMI_AUTOTUNE_CACHE: read now when it exists, rewritten after each tuning
  if (const char* path = std::getenv("DFMI_AUTOTUNE_CACHE")) {
    if (*path) {
      c->cache_path = path;
      std::string err;
      if (std::ifstream(path).good() && !tune_read(c, c->cache_path, &err)) {
        g_create_err = "DFMI_AUTOTUNE_CACHE: " + err;
        delete c;
        return DF_ERR_ARG;
      }
    }
  }
  *ctx = c;
  return DF_OK;
}

df_status df_destroy(df_ctx* ctx) {
  if (!ctx) return DF_OK;
  for (auto& t : ctx->pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  delete ctx;
  return DF_OK;
}

df_status df_set_timing(df_ctx* ctx, int enable) {
  if (!ctx) return DF_ERR_ARG;
  ctx->timing = enable != 0;
  return DF_OK;
}

df_status df_timing_read(df_ctx* ctx, double* ms, int64_t* launches, int n) {
  df_ctx* c = ctx;
  if (!c) return DF_ERR_ARG;
  if (n < 0 || (n > 0 && (!ms || !launches))) return fail(c, DF_ERR_ARG, "ms and launches need n entries");
  for (int i = 0; i < n; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  for (size_t i = 0; i < c->pending.size(); ++i) {
    const auto& t = c->pending[i];
    hipError_t e = hipEventSynchronize(t.b);
    float el = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&el, t.a, t.b);
    if (e != hipSuccess) return fail(c, DF_ERR_HIP, hip_msg(e, "reading timing events"));
    if (t.kind >= 0 && t.kind < n) {
      ms[t.kind] += el;
      launches[t.kind] += 1;
    }
  }
  for (auto& t : c->pending) {
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->pending.clear();
  return DF_OK;
}

const char* df_last_error(const df_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

df_status df_set_stream(df_ctx* ctx, void* stream) {
  if (!ctx) return DF_ERR_ARG;
  ctx->stream = (hipStream_t)stream;
  return DF_OK;
}

df_status df_set_workspace(df_ctx* ctx, void* ptr, size_t bytes) {
  if (!ctx) return DF_ERR_ARG;
  if ((ptr == nullptr) != (bytes == 0)) return fail(ctx, DF_ERR_ARG, "workspace pointer and size disagree");
  if (((uintptr_t)ptr) % kAlign != 0) return fail(ctx, DF_ERR_ARG, "workspace must be 256-byte aligned");
  ctx->ws = (char*)ptr;
  ctx->ws_bytes = bytes;
  return DF_OK;
}

}  // extern "C"

namespace {

// Workspace bytes of `op` for the sizes in *d; `limit` bounds DF_OP_STEP_BACKWARD (0: none).
df_status workspace_bytes(df_op op, const df_dims* d, size_t limit, size_t* bytes) {
  *bytes = 0;
  if (op == DF_OP_SPLIT_MATMUL) {
    if (d->m < 0 || d->n < 0 || d->k < 1 || d->nslice < 4 || d->nslice > 8) return DF_ERR_SHAPE;
    Plan pm;
    plan_split_mm(pm, d->m, d->n, d->k, d->nslice);
    *bytes = pm.total;
    return DF_OK;
  }
  if (d->naux < 1 || d->nao < 1 || d->nao > kMaxNao) return DF_ERR_SHAPE;
  if (d->ndm < 0 || d->nocc < 0 || d->nac < 0 || d->np < 0 || d->nq < 0 || d->ncol < 0 || d->n2 < 0)
    return DF_ERR_SHAPE;
  const bool split_flag = (d->flags & DF_PREC_SPLIT) != 0;
  if ((split_flag || op == DF_OP_STEP_SPLIT || op == DF_OP_STEP_BACKWARD_SPLIT) && (d->nslice < 4 || d->nslice > 8))
    return DF_ERR_SHAPE;
  Plan pl;
  switch (op) {
    case DF_OP_HALF_TRANSFORM: plan_half(pl, d->naux, d->nao, d->ncol, d->n2, d->flags, d->nslice); break;
    case DF_OP_JK:
      plan_jk(pl, d->naux, d->nao, std::max<int64_t>(d->ndm, 1), d->nocc, (d->flags & DF_WEIGHTED) != 0, d->flags,
              d->nslice);
      break;
    case DF_OP_ACTIVE_ERI: plan_act(pl, d->naux, d->nao, d->nac, d->flags, d->nslice); break;
    case DF_OP_PAPA: plan_papa(pl, d->naux, d->nao, d->nac, d->np, d->nq, d->flags, d->nslice); break;
    case DF_OP_BUILD_CHOLESKY: plan_build(pl, d->naux, d->nao); break;
    case DF_OP_EMBED_CHOLESKY: plan_embed(pl, d->naux, d->nao, d->ncol); break;
    case DF_OP_PPAA:
      plan_ppaa(pl, d->naux, d->nao, d->nac, d->nq > 0 ? d->nq : d->np);
      break;
    case DF_OP_STEP:
      plan_step(pl, d->naux, d->nao, d->nocc, d->nac, d->np, (d->flags & DF_CALLER_X) != 0);
      break;
    case DF_OP_STEP_BACKWARD: {
      const int64_t rows = backward_rows(d->naux, d->nao, d->nocc, d->nac, d->flags, limit);
      if (rows == 0) return DF_ERR_WORKSPACE;
      plan_backward(pl, d->naux, d->nao, d->nocc, d->nac, d->flags, rows);
      break;
    }
    case DF_OP_STEP_SPLIT:
      plan_step_split(pl, d->naux, d->nao, d->nocc, d->nac, d->np, d->nslice, (d->flags & DF_CALLER_X) != 0);
      break;
    case DF_OP_STEP_BACKWARD_SPLIT:
      plan_backward_split(pl, d->naux, d->nao, d->nocc, d->nac, d->flags, d->nslice);
      break;
    default: return DF_ERR_UNSUPPORTED;
  }
  *bytes = pl.total;
  return DF_OK;
}

}  // namespace

extern "C" {

df_status df_workspace_size(df_op op, const df_dims* d, size_t* bytes) {
  if (!d || !bytes) return DF_ERR_ARG;
  return workspace_bytes(op, d, 0, bytes);
}

df_status df_workspace_query(df_ctx* ctx, df_op op, const df_dims* d, size_t* bytes) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (!d || !bytes) return fail(c, DF_ERR_ARG, "dims and bytes are required");
  df_dims e = *d;
  if ((e.flags & DF_PREC_SPLIT) && e.nslice == 0) e.nslice = c->nslice;
  const df_status st = workspace_bytes(op, &e, c->scratch_limit, bytes);
  if (st == DF_ERR_WORKSPACE)
    return fail(c, st, "the scratch limit of " + std::to_string(c->scratch_limit) +
                           " bytes is below the workspace of one auxiliary row per chunk");
  if (st != DF_OK) return fail(c, st, "df_workspace_query: bad sizes or operation");
  return DF_OK;
}

df_status df_set_scratch_limit(df_ctx* ctx, size_t bytes) {
  if (!ctx) return DF_ERR_ARG;
  ctx->scratch_limit = bytes;
  return DF_OK;
}

df_status df_backward_chunk(df_ctx* ctx, const df_dims* d, int64_t* rows) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (!d || !rows) return fail(c, DF_ERR_ARG, "dims and rows are required");
  if (d->naux < 1 || d->nao < 1 || d->nao > kMaxNao || d->nocc < 0 || d->nac < 0)
    return fail(c, DF_ERR_SHAPE, "bad sizes");
  *rows = backward_rows(d->naux, d->nao, d->nocc, d->nac, d->flags, c->scratch_limit);
  if (*rows == 0) return fail(c, DF_ERR_WORKSPACE, "the scratch limit is below the workspace of one auxiliary row");
  return DF_OK;
}

df_status df_set_split_slices(df_ctx* ctx, int nslice) {
  if (!ctx) return DF_ERR_ARG;
  if (nslice < 4 || nslice > 8) return fail(ctx, DF_ERR_SHAPE, "nslice must be in [4, 8]");
  ctx->nslice = nslice;
  return DF_OK;
}

df_status df_register_split(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, const int8_t* Bs, const int* Be,
                            int nslice) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (!B) return fail(c, DF_ERR_ARG, "B is NULL");
  if (naux < 1 || nao < 1 || nao > kMaxNao) return fail(c, DF_ERR_SHAPE, "bad naux or nao");
  if (nslice < 4 || nslice > 8) return fail(c, DF_ERR_SHAPE, "nslice must be in [4, 8]");
  if (dfk::rpad32(naux * nao) > 0x7fffffffLL) return fail(c, DF_ERR_SHAPE, "naux * nao must be below 2^31 - 32");
  auto& v = c->splits;
  auto it = std::find_if(v.begin(), v.end(), [&](const df_ctx::SplitReg& r) {
    return r.B == B && r.naux == naux && r.nao == nao && r.nslice == nslice;
  });
  if (!Bs) {
    if (it != v.end()) v.erase(it);
    return DF_OK;
  }
  if (!Be) return fail(c, DF_ERR_ARG, "Be is NULL");
  if ((uintptr_t)Bs % 16 != 0) return fail(c, DF_ERR_ARG, "Bs must be 16-byte aligned");
  const df_ctx::SplitReg r{B, naux, nao, Bs, Be, nslice};
  if (it != v.end()) {
    *it = r;
    return DF_OK;
  }
  if (v.size() >= 16) return fail(c, DF_ERR_ARG, "at most 16 splits can be registered");
  v.push_back(r);
  return DF_OK;
}

df_status df_half_transform(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, const double* C,
                            int64_t ncol, double* X, const double* C2, int64_t n2, double* Y, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (df_status s = check_core(c, B, naux, nao)) return s;
  if (flags & ~(DF_ACCUMULATE | DF_PREC_SPLIT)) return fail(c, DF_ERR_UNSUPPORTED, "df_half_transform: unknown flags");
  if (!C || !X) return fail(c, DF_ERR_ARG, "C and X are required");
  if (ncol < 1) return fail(c, DF_ERR_SHAPE, "ncol must be >= 1");
  if ((C2 == nullptr) != (Y == nullptr)) return fail(c, DF_ERR_ARG, "C2 and Y must be given together");
  if (C2 && n2 < 1) return fail(c, DF_ERR_SHAPE, "n2 must be >= 1 when C2 is given");
  if (!C2 && n2 != 0) return fail(c, DF_ERR_SHAPE, "n2 must be 0 without C2");
  const bool acc = flags & DF_ACCUMULATE, sp = flags & DF_PREC_SPLIT;
  const int64_t npair = nao * (nao + 1) / 2;
  std::vector<Range> rs = {{B, dbytes(naux * npair), "B", false},
                           {C, dbytes(nao * ncol), "C", false},
                           {X, dbytes(naux * nao * ncol), "X", true},
                           {C2, dbytes(nao * n2), "C2", false},
                           {Y, dbytes(naux * n2 * ncol), "Y", true}};
  const df_ctx::SplitReg* reg = nullptr;
  if (sp)
    if (df_status s = split_for_call(c, B, naux, nao, naux * std::max<int64_t>(ncol, n2), &reg, rs)) return s;
  Plan pl;
  const HalfPlan p = plan_half(pl, naux, nao, ncol, n2, flags, c->nslice);
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = need_ws(c, pl.total)) return s;
  rs.push_back({c->ws, pl.total, "workspace", true});
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = enter(c)) return s;
  char* ws = c->ws;
  // this call's X: into X itself, or, when it must be added to X and also feed Y, into xnew first
  double* Xd = acc && C2 ? (double*)(ws + p.xnew) : X;
  const int xacc = acc && !C2;
  if (!sp) {
    double* cpad = (double*)(ws + p.cpad);
    const ColBlock blk{C, ncol, ncol, 0};
    if (df_status s = pad_operand(c, cpad, nao, ncol, &blk, 1)) return s;
    dfk::OutMap OX = out_pmajor(Xd, naux, nao, ncol, ncol);
    OX.accumulate = xacc;
    if (df_status s = run_half(c, B, naux, nao, cpad, ncol, OX)) return s;
    if (C2)
      if (df_status s = run_mo_pmajor(c, C2, n2, Xd, naux, nao, ncol, Y, acc)) return s;
  } else {
    // rows (P, mu) of b^P against the rows c of C, both over nu
    const SplitOp cs = split_in(ws, p.cs);
    if (df_status s = split_of(c, dfk::op_map(C, ncol, 1, nao, ncol), nao, c->nslice, cs)) return s;
    dfk::OutMap OX = dfk::out_plain(Xd, naux * nao, ncol, ncol);
    OX.accumulate = xacc;
    if (df_status s = split_half(c, *reg, cs, ncol, OX)) return s;
    if (C2) {
      // Y[P][p][c] = sum_mu C2[mu][p] X[P][mu][c]: rows p of C2 against rows (P, c) of X, over mu
      dfk::OpMap ox = dfk::op_map(Xd, naux * ncol, 1, nao, ncol);
      ox.rl = ncol;
      ox.s_rh = nao * ncol;
      const SplitOp xs = split_in(ws, p.xs), c2s = split_in(ws, p.c2s);
      if (df_status s = split_of(c, ox, nao, c->nslice, xs)) return s;
      if (df_status s = split_of(c, dfk::op_map(C2, n2, 1, nao, n2), nao, c->nslice, c2s)) return s;
      dfk::OutMap O = dfk::out_plain(Y, n2, naux * ncol, ncol);
      O.nl = ncol;
      O.s_nh = n2 * ncol;
      O.accumulate = acc;
      if (df_status s = slice_product(c, DF_KERNEL_MO_TRANSFORM, c2s, n2, xs, naux * ncol, nao, c->nslice, O)) return s;
    }
  }
  if (acc && C2) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_add(Xd, naux * nao * ncol, X, c->stream), "add launch");
  return DF_OK;
}

// The JK call on workspace `ws` laid out by plan p (already checked): X of the densities, v of
// this call (row stride ldv in v), J and K.  acc_jk adds J and K to the outputs, acc_v adds v; v of
// this call alone feeds J.  reg: the registered planes of B (split precision) or null (FP64).
static df_status jk_run(df_ctx* c, char* ws, const JkPlan& p, const double* B, int64_t naux, int64_t nao, int64_t ndm,
                        const double* Cocc, int64_t nocc, const double* w, double* J, double* K, double* v,
                        int64_t ldv, bool acc_jk, bool acc_v, const df_ctx::SplitReg* reg) {
  const bool sp = reg != nullptr;
  const int64_t ncol = ndm * nocc;
  double* X = (double*)(ws + p.x);
  if (!sp) {
    double* cc = (double*)(ws + p.ccat);
    std::vector<ColBlock> blks((size_t)ndm);
    for (int64_t z = 0; z < ndm; ++z) blks[(size_t)z] = ColBlock{Cocc + z * nao * nocc, nocc, nocc, z * nocc};
    if (df_status s = pad_operand(c, cc, nao, ncol, blks.data(), (int)ndm)) return s;
    if (df_status s = run_half(c, B, naux, nao, cc, ncol, out_pmajor(X, naux, nao, ncol, ncol))) return s;
  } else {
    // the rows (z, c) of the factors over mu, then X[P][mu][(z, c)] from the planes of b^P
    dfk::OpMap oc = dfk::op_map(Cocc, ncol, 1, nao, nocc);
    oc.rl = nocc;
    oc.s_rh = nao * nocc;
    const SplitOp cs = split_in(ws, p.cs);
    if (df_status s = split_of(c, oc, nao, c->nslice, cs)) return s;
    if (df_status s = split_half(c, *reg, cs, ncol, dfk::out_plain(X, naux * nao, ncol, ncol))) return s;
  }
  if (J || v) {
    // v of this call (into v itself unless it is to be added to v)
    const bool direct = v && !acc_v;
    double* vv = direct ? v : (double*)(ws + p.vtmp);
    const int64_t ldvv = direct ? ldv : naux;
    DF_LAUNCH(DF_KERNEL_JVEC, dfk::launch_jvec(X, naux, nao, ncol, Cocc, w, nocc, ndm, vv, c->stream, 0, ldvv),
              "J-vector launch");
    if (J)
      DF_LAUNCH(DF_KERNEL_COULOMB, dfk::launch_coulomb(B, naux, nao, vv, ndm, J, c->stream, acc_jk, ldvv),
                "Coulomb launch");
    if (v && acc_v)
      DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_copy_rows(vv, ndm, naux, v, ldv, 1, c->stream), "add launch");
  }
  if (K) {
    double* kpart = (double*)(ws + p.kpart);
    if (!sp) {
      if (df_status s = run_k(c, X, w, naux, nao, ncol, nocc, ndm, p.nsplit, kpart, K, acc_jk)) return s;
    } else {
      // K_z = sum_{P, c} X[P][m][(z, c)] w_zc X[P][n][(z, c)]: the rows m of each density's X_occ
      // over (P, c), against those of X diag(w) when there are weights; lower tiles, reduced and
      // mirrored
      const SplitOp xo = split_in(ws, p.xos), xw = split_in(ws, p.xws);
      const double* Xw = X;
      if (w) {
        Xw = (double*)(ws + p.xw);
        DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_scale_cols(X, naux * nao * ncol, ncol, w, (double*)Xw, c->stream),
                  "scale launch");
      }
      for (int64_t z = 0; z < ndm; ++z) {
        for (int side = 0; side < (w ? 2 : 1); ++side) {
          dfk::OpMap ox = dfk::op_map((side ? Xw : X) + z * nocc, nao, ncol, nocc, 1);
          ox.kb_n = naux;
          ox.s_kb = nao * ncol;
          const SplitOp d = side ? xw : xo;
          if (df_status s = split_of(c, ox, naux * nocc, c->nslice, SplitOp{d.planes + z * p.xplane, d.ex + z * nao}))
            return s;
        }
      }
      const SplitOp rb = w ? xw : xo;
      const dfk::SliceBatch zs{p.xplane, nao, p.xplane, nao};
      DF_LAUNCH(DF_KERNEL_K_SYRK,
                dfk::launch_slice_gemm_batched(xo.planes, xo.ex, nao, rb.planes, rb.ex, nao, dfk::kpad64(naux * nocc),
                                               c->nslice, dfk::out_plain(kpart, nao, nao, nao), true, p.nsplit, kpart,
                                               ndm, zs, c->stream),
                "slice product launch");
      DF_LAUNCH(DF_KERNEL_K_REDUCE, dfk::launch_syrk_reduce(kpart, p.nsplit, nao, ndm, K, c->stream, acc_jk),
                "K reduce launch");
    }
  }
  return DF_OK;
}

// Arguments of the JK call shared by df_jk and df_jk_noalloc; fills the ranges it reads and writes.
static df_status jk_check(df_ctx* c, const double* B, int64_t naux, int64_t nao, int64_t ndm, const double* Cocc,
                          int64_t nocc, const double* w, double* J, double* K, double* v, std::vector<Range>& rs) {
  if (df_status s = check_core(c, B, naux, nao)) return s;
  if (ndm < 1 || ndm > 65535) return fail(c, DF_ERR_SHAPE, "ndm must be in [1, 65535]");
  if (nocc < 0) return fail(c, DF_ERR_SHAPE, "nocc must be >= 0");
  if (nocc > 0 && !Cocc) return fail(c, DF_ERR_ARG, "Cocc is NULL");
  const int64_t npair = nao * (nao + 1) / 2;
  rs = {{B, dbytes(naux * npair), "B", false},
        {Cocc, dbytes(ndm * nao * nocc), "Cocc", false},
        {w, dbytes(ndm * nocc), "w", false},
        {J, dbytes(ndm * nao * nao), "J", true},
        {K, dbytes(ndm * nao * nao), "K", true},
        {v, dbytes(ndm * naux), "v", true}};
  return DF_OK;
}

// nocc = 0: every output is zero (or, accumulating, unchanged)
static df_status jk_empty(df_ctx* c, int64_t naux, int64_t nao, int64_t ndm, double* J, double* K, double* v,
                          bool acc) {
  if (acc) return DF_OK;
  if (J) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(J, ndm * nao * nao, c->stream), "fill");
  if (K) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(K, ndm * nao * nao, c->stream), "fill");
  if (v) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(v, ndm * naux, c->stream), "fill");
  return DF_OK;
}

df_status df_jk(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, int64_t ndm, const double* Cocc,
                int64_t nocc, const double* w, double* J, double* K, double* v, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (flags & ~(DF_ACCUMULATE | DF_PREC_SPLIT)) return fail(c, DF_ERR_UNSUPPORTED, "df_jk: unknown flags");
  std::vector<Range> rs;
  if (df_status s = jk_check(c, B, naux, nao, ndm, Cocc, nocc, w, J, K, v, rs)) return s;
  const bool acc = flags & DF_ACCUMULATE, sp = flags & DF_PREC_SPLIT;
  const int64_t ncol = ndm * nocc;
  const bool work = nocc > 0 && (J || K || v);
  const df_ctx::SplitReg* reg = nullptr;
  if (sp && work) {
    if (df_status s = split_for_call(c, B, naux, nao, std::max(ncol, nao), &reg, rs)) return s;
    if (naux * nocc > (int64_t(1) << 30)) return fail(c, DF_ERR_SHAPE, "naux * nocc too large for the split path");
  }
  Plan pl;
  const JkPlan p = plan_jk(pl, naux, nao, ndm, nocc, w != nullptr, flags, c->nslice);
  if (work) {
    if (!check_overlap(c, rs)) return DF_ERR_ARG;
    if (df_status s = need_ws(c, pl.total)) return s;
    rs.push_back({c->ws, pl.total, "workspace", true});
  }
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (nocc == 0 && acc) return DF_OK;   // nothing to add
  if (df_status s = enter(c)) return s;
  if (nocc == 0) return jk_empty(c, naux, nao, ndm, J, K, v, acc);
  if (!work) return DF_OK;
  return jk_run(c, c->ws, p, B, naux, nao, ndm, Cocc, nocc, w, J, K, v, naux, acc, acc, reg);
}

// Address of the static scratch on the context's device (current after enter()), looked up once
// per device.
static df_status scratch_address(df_ctx* c, char** addr) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(c->device);
  if (it != g_scratch_addr.end()) {
    *addr = it->second;
    return DF_OK;
  }
  void* ptr = nullptr;
  DF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
  if (!ptr || (uintptr_t)ptr % kAlign != 0) return fail(c, DF_ERR_HIP, "the static scratch has no aligned address");
  g_scratch_addr[c->device] = (char*)ptr;
  *addr = (char*)ptr;
  return DF_OK;
}

df_status df_jk_noalloc(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, int64_t ndm, const double* Cocc,
                        int64_t nocc, const double* w, double* J, double* K, double* v, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (flags & ~DF_ACCUMULATE) return fail(c, DF_ERR_UNSUPPORTED, "df_jk_noalloc takes DF_ACCUMULATE only");
  std::vector<Range> rs;
  if (df_status s = jk_check(c, B, naux, nao, ndm, Cocc, nocc, w, J, K, v, rs)) return s;
  const bool acc = flags & DF_ACCUMULATE;
  const bool work = nocc > 0 && (J || K || v);
  int64_t rows = 0;
  if (work) {
    rows = noalloc_jk_rows(naux, nao, ndm, nocc, w != nullptr);
    if (rows == 0)
      return fail(c, DF_ERR_WORKSPACE, "df_jk_noalloc: one auxiliary row needs more than the " +
                                           std::to_string(kNoallocBytes >> 20) + " MiB static scratch");
  }
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (nocc == 0 && acc) return DF_OK;
  if (df_status s = enter(c)) return s;
  if (nocc == 0) return jk_empty(c, naux, nao, ndm, J, K, v, acc);
  if (!work) return DF_OK;
  char* ws = nullptr;
  if (df_status s = scratch_address(c, &ws)) return s;
  // no timing events here: the first ones of a context would be created (allocated) on demand
  const bool timing = c->timing;
  c->timing = false;
  const int64_t npair = nao * (nao + 1) / 2;
  const int nsplit = noalloc_jk_splits(nao, rows, ndm);
  df_status st = DF_OK;
  for (int64_t p0 = 0; p0 < naux && st == DF_OK; p0 += rows) {
    const int64_t r = std::min(rows, naux - p0);
    Plan pl;
    const JkPlan p = plan_jk(pl, r, nao, ndm, nocc, w != nullptr, 0, c->nslice, nsplit);
    // J and K add up over the blocks; each block writes its own columns of v
    st = jk_run(c, ws, p, B + p0 * npair, r, nao, ndm, Cocc, nocc, w, J, K, v ? v + p0 : nullptr, naux,
                acc || p0 > 0, acc, nullptr);
  }
  c->timing = timing;
  return st;
}

// b^P_{lu} = sum_mu Cl[mu][l] X^act[mu][P][u] for every P into out [naux][nl][nac], from int8
// slices: the rows l of Cl (planes ls, written here unless `have_ls`) against the rows (P, u) of
// X_act (planes xas), both over mu.
static df_status split_second(df_ctx* c, const double* Cl, int64_t nl, SplitOp ls, SplitOp xas, int64_t naux,
                              int64_t nao, int64_t nac, double* out, bool have_ls = false) {
  if (!have_ls)
    if (df_status s = split_of(c, dfk::op_map(Cl, nl, 1, nao, nl), nao, c->nslice, ls)) return s;
  dfk::OutMap O = dfk::out_plain(out, nl, naux * nac, nac);
  O.nl = nac;
  O.s_nh = nl * nac;
  return slice_product(c, DF_KERNEL_MO_TRANSFORM, ls, nl, xas, naux * nac, nao, c->nslice, O);
}

// X_act AO-major [nao][naux][nac] from the registered planes of B (planes cas of the rows of Cact
// written first), and the planes xas of its rows (P, u) over mu.
static df_status split_xact(df_ctx* c, const df_ctx::SplitReg& r, const double* Cact, int64_t nac, double* X,
                            SplitOp cas, SplitOp xas) {
  const int64_t naux = r.naux, nao = r.nao;
  if (df_status s = split_of(c, dfk::op_map(Cact, nac, 1, nao, nac), nao, c->nslice, cas)) return s;
  dfk::OutMap OX = dfk::out_plain(X, naux * nao, nac, naux * nac);
  OX.ml = nao;   // row (P, mu) at P * nac + mu * naux * nac
  OX.s_mh = nac;
  if (df_status s = split_half(c, r, cas, nac, OX)) return s;
  return split_of(c, dfk::op_map(X, naux * nac, 1, nao, naux * nac), nao, c->nslice, xas);
}

df_status df_active_eri(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, const double* Cact, int64_t nac,
                        double* eri, double* buv, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (df_status s = check_core(c, B, naux, nao)) return s;
  if (flags & ~(DF_ACCUMULATE | DF_PREC_SPLIT)) return fail(c, DF_ERR_UNSUPPORTED, "df_active_eri: unknown flags");
  if (nac < 0) return fail(c, DF_ERR_SHAPE, "nac must be >= 0");
  if (nac > 0 && (!Cact || !eri)) return fail(c, DF_ERR_ARG, "Cact and eri are required");
  const bool acc = flags & DF_ACCUMULATE, sp = flags & DF_PREC_SPLIT;
  const int64_t npair = nao * (nao + 1) / 2, n2 = nac * nac;
  std::vector<Range> rs = {{B, dbytes(naux * npair), "B", false},
                           {Cact, dbytes(nao * nac), "Cact", false},
                           {eri, dbytes(n2 * n2), "eri", true},
                           {buv, dbytes(naux * n2), "buv", true}};
  const df_ctx::SplitReg* reg = nullptr;
  if (sp && nac > 0)
    if (df_status s = split_for_call(c, B, naux, nao, naux * nac, &reg, rs)) return s;
  Plan pl;
  const ActPlan p = plan_act(pl, naux, nao, nac, flags, c->nslice);
  if (nac > 0) {
    if (!check_overlap(c, rs)) return DF_ERR_ARG;
    if (df_status s = need_ws(c, pl.total)) return s;
    rs.push_back({c->ws, pl.total, "workspace", true});
  }
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (nac == 0) return DF_OK;
  if (df_status s = enter(c)) return s;
  char* ws = c->ws;
  double* X = (double*)(ws + p.x);
  double* bu = buv && !acc ? buv : (double*)(ws + p.buv);   // b_uv of this call
  if (!sp) {
    double* cpad = (double*)(ws + p.cpad);
    const ColBlock blk{Cact, nac, nac, 0};
    if (df_status s = pad_operand(c, cpad, nao, nac, &blk, 1)) return s;
    if (df_status s = run_half(c, B, naux, nao, cpad, nac, out_split(nullptr, X, naux, nao, 0, nac))) return s;
    if (df_status s = run_mo(c, Cact, nac, X, naux, nao, nac, bu)) return s;
    if (df_status s = run_pgemm(c, DF_KERNEL_ERI, bu, n2, bu, n2, naux, eri, acc)) return s;
  } else {
    const SplitOp cas = split_in(ws, p.cas), xas = split_in(ws, p.xas), bvs = split_in(ws, p.buvs);
    if (df_status s = split_xact(c, *reg, Cact, nac, X, cas, xas)) return s;
    // b_uv: the planes of Cact's rows are already there
    dfk::OutMap O = dfk::out_plain(bu, nac, naux * nac, nac);
    O.nl = nac;
    O.s_nh = n2;
    if (df_status s = slice_product(c, DF_KERNEL_MO_TRANSFORM, cas, nac, xas, naux * nac, nao, c->nslice, O)) return s;
    if (df_status s = split_of(c, dfk::op_map(bu, n2, 1, naux, n2), naux, c->nslice, bvs)) return s;
    dfk::OutMap Oe = dfk::out_plain(eri, n2, n2, n2);
    Oe.accumulate = acc;
    if (df_status s = slice_product(c, DF_KERNEL_ERI, bvs, n2, bvs, n2, naux, c->nslice, Oe)) return s;
  }
  if (buv && acc) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_add(bu, naux * n2, buv, c->stream), "add launch");
  return DF_OK;
}

df_status df_papa(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, const double* Cp, int64_t np,
                  const double* Cact, int64_t nac, const double* Cq, int64_t nq, double* out, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (df_status s = check_core(c, B, naux, nao)) return s;
  if (flags & ~(DF_PAPA_FULL | DF_ACCUMULATE | DF_PREC_SPLIT)) return fail(c, DF_ERR_UNSUPPORTED, "unknown flag bits");
  const bool full = flags & DF_PAPA_FULL, acc = flags & DF_ACCUMULATE, sp = flags & DF_PREC_SPLIT;
  if (np < 0 || nac < 0 || nq < 0) return fail(c, DF_ERR_SHAPE, "sizes must be >= 0");
  if (full) {
    if (nq > 0 && !Cq) return fail(c, DF_ERR_ARG, "DF_PAPA_FULL needs Cq");
  } else {
    if (Cq || nq != 0) return fail(c, DF_ERR_ARG, "Cq/nq are only used with DF_PAPA_FULL");
  }
  const int64_t nout = full ? np * nac * nq * nac : np * nac * nac * nac;
  if (nout > 0 && (!Cp || !Cact || !out)) return fail(c, DF_ERR_ARG, "Cp, Cact and out are required");
  const int64_t npair = nao * (nao + 1) / 2;
  std::vector<Range> rs = {{B, dbytes(naux * npair), "B", false},
                           {Cp, dbytes(nao * np), "Cp", false},
                           {Cact, dbytes(nao * nac), "Cact", false},
                           {Cq, dbytes(nao * nq), "Cq", false},
                           {out, dbytes(nout), "out", true}};
  const df_ctx::SplitReg* reg = nullptr;
  if (sp && nout > 0)
    if (df_status s = split_for_call(c, B, naux, nao, naux * nac, &reg, rs)) return s;
  if (sp && nout > 0 && !split_sizes_ok(naux, nao, std::max(np, nq) * nac))
    return fail(c, DF_ERR_SHAPE, "problem too large for the split path");
  Plan pl;
  const PapaPlan p = plan_papa(pl, naux, nao, nac, np, nq, flags, c->nslice);
  if (nout > 0) {
    if (!check_overlap(c, rs)) return DF_ERR_ARG;
    if (df_status s = need_ws(c, pl.total)) return s;
    rs.push_back({c->ws, pl.total, "workspace", true});
  }
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (nout == 0) return DF_OK;
  if (df_status s = enter(c)) return s;
  char* ws = c->ws;
  double* X = (double*)(ws + p.x);
  double* bpu = (double*)(ws + p.bpu);
  // the right-hand factor: b_vw (default) or b_qv (DF_PAPA_FULL), [naux][nr][nac]
  const double* Cr = full ? Cq : Cact;
  const int64_t nr = full ? nq : nac;
  double* br = (double*)(ws + (full ? p.bqv : p.bvw));
  if (!sp) {
    double* cpad = (double*)(ws + p.cpad);
    const ColBlock blk{Cact, nac, nac, 0};
    if (df_status s = pad_operand(c, cpad, nao, nac, &blk, 1)) return s;
    if (df_status s = run_half(c, B, naux, nao, cpad, nac, out_split(nullptr, X, naux, nao, 0, nac))) return s;
    if (df_status s = run_mo(c, Cp, np, X, naux, nao, nac, bpu)) return s;
    if (df_status s = run_mo(c, Cr, nr, X, naux, nao, nac, br)) return s;
    return run_pgemm(c, DF_KERNEL_PAPA, bpu, np * nac, br, nr * nac, naux, out, acc);
  }
  const SplitOp xas = split_in(ws, p.xas), cps = split_in(ws, p.cps), bps = split_in(ws, p.bpus);
  const SplitOp cas = split_in(ws, p.cas), crs = full ? split_in(ws, p.cqs) : cas;
  const SplitOp brs = split_in(ws, full ? p.bqvs : p.bvws);
  if (df_status s = split_xact(c, *reg, Cact, nac, X, cas, xas)) return s;
  if (df_status s = split_second(c, Cp, np, cps, xas, naux, nao, nac, bpu)) return s;
  // the default form's right factor b_vw uses the planes of Cact's rows made for X_act
  if (df_status s = split_second(c, Cr, nr, crs, xas, naux, nao, nac, br, !full)) return s;
  if (df_status s = split_of(c, dfk::op_map(bpu, np * nac, 1, naux, np * nac), naux, c->nslice, bps)) return s;
  if (df_status s = split_of(c, dfk::op_map(br, nr * nac, 1, naux, nr * nac), naux, c->nslice, brs)) return s;
  dfk::OutMap O = dfk::out_plain(out, np * nac, nr * nac, nr * nac);
  O.accumulate = acc;
  return slice_product(c, DF_KERNEL_PAPA, bps, np * nac, brs, nr * nac, naux, c->nslice, O);
}

// (pq|uv) into out [nuv][np][nq] with the workspace pieces of p at ws (see plan_ppaa)
static df_status ppaa_run(df_ctx* c, char* ws, const PpaaPlan& p, const double* B, int64_t naux, int64_t nao,
                          const double* Cp, int64_t np, const double* Cq, int64_t nq, const double* Cact,
                          int64_t nac, double* out) {
  const int64_t npair = nao * (nao + 1) / 2, nuv = nac * (nac + 1) / 2;
  double* X = (double*)(ws + p.x);
  double* buv = (double*)(ws + p.buv);
  double* vp = (double*)(ws + p.vp);
  double* W = (double*)(ws + p.w);
  double* T = (double*)(ws + p.t);
  double* cpa = (double*)(ws + p.cpa);
  double* cpq = (double*)(ws + p.cpq);
  // b^P_uv for every P, its lower triangle packed: vp [naux][nuv]
  const ColBlock ba{Cact, nac, nac, 0};
  if (df_status s = pad_operand(c, cpa, nao, nac, &ba, 1)) return s;
  if (df_status s = run_half(c, B, naux, nao, cpa, nac, out_split(nullptr, X, naux, nao, 0, nac))) return s;
  if (df_status s = run_mo(c, Cact, nac, X, naux, nao, nac, buv)) return s;
  DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_pack_lower(buv, naux, nac, vp, c->stream), "pack launch");
  const ColBlock bq{Cq, nq, nq, 0};
  if (df_status s = pad_operand(c, cpq, nao, nq, &bq, 1)) return s;
  // P ranges whose packed rows stay inside 31-bit offsets
  const int64_t pb = std::max<int64_t>(1, ((int64_t(1) << 31) - 1) / npair);
  for (int64_t u0 = 0; u0 < nuv; u0 += p.chunk) {
    const int64_t zc = std::min<int64_t>(p.chunk, nuv - u0);
    // W_uv = sum_P b^P_uv b^P over the packed pairs
    for (int64_t p0 = 0; p0 < naux; p0 += pb) {
      const int64_t pn = std::min<int64_t>(pb, naux - p0);
      const dfk::OpMap A = dfk::op_map(vp + p0 * nuv + u0, zc, 1, pn, nuv);
      const dfk::OpMap Bm = dfk::op_map(B + p0 * npair, npair, 1, pn, npair);
      dfk::OutMap O = dfk::out_plain(W, zc, npair, npair);
      O.accumulate = p0 > 0;
      DF_LAUNCH(DF_KERNEL_PAPA, dfk::launch_gemm(A, Bm, O, 1, c->stream), "W product launch");
    }
    // T_uv = W_uv Cq (W_uv read packed), then out[uv] = Cp^T T_uv
    if (df_status s = run_half(c, W, zc, nao, cpq, nq, out_pmajor(T, zc, nao, nq, nq))) return s;
    if (df_status s = run_mo_pmajor(c, Cp, np, T, zc, nao, nq, out + u0 * np * nq)) return s;
  }
  return DF_OK;
}

df_status df_ppaa(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, const double* Cp, int64_t np,
                  const double* Cq, int64_t nq, const double* Cact, int64_t nac, double* out, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (df_status s = check_core(c, B, naux, nao)) return s;
  if (flags != 0) return fail(c, DF_ERR_UNSUPPORTED, "df_ppaa takes no flags");
  if (np < 0 || nac < 0 || nq < 0) return fail(c, DF_ERR_SHAPE, "sizes must be >= 0");
  if (!Cq) {
    if (nq != 0) return fail(c, DF_ERR_ARG, "nq must be 0 when Cq is NULL (Cq = Cp)");
    Cq = Cp;
    nq = np;
  }
  const int64_t nuv = nac * (nac + 1) / 2, nout = nuv * np * nq;
  if (nout > 0 && (!Cp || !Cact || !out)) return fail(c, DF_ERR_ARG, "Cp, Cact and out are required");
  const int64_t npair = nao * (nao + 1) / 2;
  std::vector<Range> rs = {{B, dbytes(naux * npair), "B", false},
                           {Cp, dbytes(nao * np), "Cp", false},
                           {Cq == Cp ? nullptr : Cq, dbytes(nao * nq), "Cq", false},
                           {Cact, dbytes(nao * nac), "Cact", false},
                           {out, dbytes(nout), "out", true}};
  Plan pl;
  const PpaaPlan p = plan_ppaa(pl, naux, nao, nac, nq);
  if (nout > 0) {
    if (!check_overlap(c, rs)) return DF_ERR_ARG;
    if (df_status s = need_ws(c, pl.total)) return s;
    rs.push_back({c->ws, pl.total, "workspace", true});
  }
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (nout == 0) return DF_OK;
  if (df_status s = enter(c)) return s;
  return ppaa_run(c, c->ws, p, B, naux, nao, Cp, np, Cq, nq, Cact, nac, out);
}

df_status df_build_cholesky(df_ctx* ctx, const double* metric, const double* eri3, int64_t naux, int64_t nao,
                            double* L, double* B, int* info, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (flags != 0) return fail(c, DF_ERR_UNSUPPORTED, "df_build_cholesky takes no flags");
  if (!metric || !eri3 || !L || !B || !info) return fail(c, DF_ERR_ARG, "metric, eri3, L, B and info are required");
  if (naux < 1 || nao < 1) return fail(c, DF_ERR_SHAPE, "naux and nao must be >= 1");
  const int64_t nb = dfk::kCholNB, npair = nao * (nao + 1) / 2;
  // a block row of the substitution is addressed with 32-bit offsets
  if (nb * npair >= (int64_t(1) << 32) || naux * naux >= (int64_t(1) << 32))
    return fail(c, DF_ERR_SHAPE, "nao or naux too large for df_build_cholesky");
  // L may be the metric itself and B the integrals themselves (in place); nothing else may overlap
  std::vector<Range> rs = {{metric == L ? nullptr : metric, dbytes(naux * naux), "metric", false},
                           {eri3 == B ? nullptr : eri3, dbytes(naux * npair), "eri3", false},
                           {L, dbytes(naux * naux), "L", true},
                           {B, dbytes(naux * npair), "B", true},
                           {info, sizeof(int), "info", true}};
  Plan pl;
  const BuildPlan p = plan_build(pl, naux, nao);
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = need_ws(c, pl.total)) return s;
  rs.push_back({c->ws, pl.total, "workspace", true});
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = enter(c)) return s;
  double* linv = (double*)(c->ws + p.linv);
  double* panel = (double*)(c->ws + p.panel);
  double* T = (double*)(c->ws + p.t);
  const int64_t n = naux;
  if (L != metric)
    DF_LAUNCH(DF_KERNEL_OTHER, hipMemcpyAsync(L, metric, dbytes(n * n), hipMemcpyDeviceToDevice, c->stream),
              "metric copy");
  // right-looking blocked Cholesky: the diagonal block of column k (all earlier updates applied)
  // is factored and inverted in one workgroup, the panel below is multiplied by the inverted
  // block, and the trailing matrix takes the panel's update as one product over the whole square
  // (its upper half is never read and is zeroed at the end)
  for (int64_t k = 0; k < p.nblk; ++k) {
    const int64_t k0 = k * nb, kb = std::min(nb, n - k0), r0 = k0 + kb, m = n - r0;
    DF_LAUNCH(DF_KERNEL_BUILD,
              dfk::launch_chol_block(L + k0 * n + k0, n, (int)kb, linv + k * nb * nb, info, k0, k == 0, c->stream),
              "diagonal block launch");
    if (m == 0) continue;
    // L_{>k,k} = A_{>k,k} L_kk^-T, through the panel buffer (the product reads the block it replaces)
    const dfk::OpMap A = dfk::op_map(L + r0 * n + k0, m, n, kb, 1);
    const dfk::OpMap Bm = dfk::op_map(linv + k * nb * nb, kb, nb, kb, 1);
    DF_LAUNCH(DF_KERNEL_BUILD, dfk::launch_gemm(A, Bm, dfk::out_plain(panel, m, kb, nb), 1, c->stream),
              "panel solve launch");
    DF_LAUNCH(DF_KERNEL_OTHER,
              hipMemcpy2DAsync(L + r0 * n + k0, n * sizeof(double), panel, nb * sizeof(double), kb * sizeof(double),
                               m, hipMemcpyDeviceToDevice, c->stream),
              "panel copy");
    // A_{>k,>k} -= L_{>k,k} L_{>k,k}^T
    dfk::OutMap O = dfk::out_plain(L + r0 * n + r0, m, m, n);
    O.alpha = -1.0;
    O.accumulate = 1;
    DF_LAUNCH(DF_KERNEL_BUILD, dfk::launch_gemm(A, A, O, 1, c->stream), "trailing update launch");
  }
  DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_zero_upper(L, n, c->stream), "zero launch");
  // forward substitution by block rows: B_k = L_kk^-1 (E_k - L_{k,<k} B_{<k})
  for (int64_t k = 0; k < p.nblk; ++k) {
    const int64_t k0 = k * nb, kb = std::min(nb, n - k0);
    DF_LAUNCH(DF_KERNEL_OTHER,
              hipMemcpyAsync(T, eri3 + k0 * npair, dbytes(kb * npair), hipMemcpyDeviceToDevice, c->stream),
              "block row copy");
    if (k0 > 0) {
      // the contraction over the k earlier (full) blocks, one 64-bit-strided slab per block
      dfk::OpMap A = dfk::op_map(L + k0 * n, kb, n, nb, 1);
      A.kb_n = k;
      A.s_kb = nb;
      dfk::OpMap Bm = dfk::op_map(B, npair, 1, nb, npair);
      Bm.kb_n = k;
      Bm.s_kb = nb * npair;
      dfk::OutMap O = dfk::out_plain(T, kb, npair, npair);
      O.alpha = -1.0;
      O.accumulate = 1;
      DF_LAUNCH(DF_KERNEL_BUILD, dfk::launch_gemm(A, Bm, O, 1, c->stream), "substitution update launch");
    }
    const dfk::OpMap A = dfk::op_map(linv + k * nb * nb, kb, nb, kb, 1);
    const dfk::OpMap Bm = dfk::op_map(T, npair, 1, kb, npair);
    DF_LAUNCH(DF_KERNEL_BUILD,
              dfk::launch_gemm(A, Bm, dfk::out_plain(B + k0 * npair, kb, npair, npair), 1, c->stream),
              "block solve launch");
  }
  return DF_OK;
}

df_status df_embed_cholesky(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, const double* M, int64_t nemb,
                            double* Be, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (df_status s = check_core(c, B, naux, nao)) return s;
  if (flags != 0) return fail(c, DF_ERR_UNSUPPORTED, "df_embed_cholesky takes no flags");
  if (nemb < 0 || nemb > kMaxNao) return fail(c, DF_ERR_SHAPE, "nemb must be in [0, 46340]");
  if (nemb > 0 && (!M || !Be)) return fail(c, DF_ERR_ARG, "M and Be are required");
  const int64_t npair = nao * (nao + 1) / 2, npe = nemb * (nemb + 1) / 2;
  std::vector<Range> rs = {{B, dbytes(naux * npair), "B", false},
                           {M, dbytes(nao * nemb), "M", false},
                           {Be, dbytes(naux * npe), "Be", true}};
  Plan pl;
  const EmbedPlan p = plan_embed(pl, naux, nao, nemb);
  if (nemb > 0) {
    if (!check_overlap(c, rs)) return DF_ERR_ARG;
    if (df_status s = need_ws(c, pl.total)) return s;
    rs.push_back({c->ws, pl.total, "workspace", true});
  }
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (nemb == 0) return DF_OK;
  if (df_status s = enter(c)) return s;
  double* mpad = (double*)(c->ws + p.mpad);
  double* X = (double*)(c->ws + p.x);
  double* Y = (double*)(c->ws + p.y);
  const ColBlock blk{M, nemb, nemb, 0};
  if (df_status s = pad_operand(c, mpad, nao, nemb, &blk, 1)) return s;
  for (int64_t p0 = 0; p0 < naux; p0 += p.chunk) {
    const int64_t pc = std::min(p.chunk, naux - p0);
    if (df_status s = run_half(c, B + p0 * npair, pc, nao, mpad, nemb, out_pmajor(X, pc, nao, nemb, nemb)))
      return s;
    if (df_status s = run_mo_pmajor(c, M, nemb, X, pc, nao, nemb, Y)) return s;
    DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_pack_lower(Y, pc, nemb, Be + p0 * npe, c->stream), "pack launch");
  }
  return DF_OK;
}

df_status df_step(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, const double* Cocc, int64_t nocc,
                  const double* w, const double* Cact, int64_t nac, const double* Cp, int64_t np, double* J,
                  double* K, double* v, double* eri, double* papa, double* Xocc, double* Xact, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (df_status s = check_core(c, B, naux, nao)) return s;
  if (flags != 0) return fail(c, DF_ERR_UNSUPPORTED, "df_step takes no flags");
  if (nocc < 0 || nac < 0 || np < 0) return fail(c, DF_ERR_SHAPE, "sizes must be >= 0");
  if (nocc > 0 && !Cocc) return fail(c, DF_ERR_ARG, "Cocc is NULL");
  if (nac > 0 && !Cact) return fail(c, DF_ERR_ARG, "Cact is NULL");
  if (np > 0 && !Cp) return fail(c, DF_ERR_ARG, "Cp is NULL");
  const bool caller_x = Xocc != nullptr || Xact != nullptr;
  if (caller_x && ((nocc > 0 && !Xocc) || (nac > 0 && !Xact)))
    return fail(c, DF_ERR_ARG, "Xocc and Xact must be given together (NULL only for an empty one)");
  const int64_t npair = nao * (nao + 1) / 2;
  std::vector<Range> rs = {{B, dbytes(naux * npair), "B", false},
                           {Cocc, dbytes(nao * nocc), "Cocc", false},
                           {w, dbytes(nocc), "w", false},
                           {Cact, dbytes(nao * nac), "Cact", false},
                           {Cp, dbytes(nao * np), "Cp", false},
                           {J, dbytes(nao * nao), "J", true},
                           {K, dbytes(nao * nao), "K", true},
                           {v, dbytes(naux), "v", true},
                           {eri, dbytes(nac * nac * nac * nac), "eri", true},
                           {papa, dbytes(np * nac * nac * nac), "papa", true},
                           {Xocc, dbytes(naux * nao * nocc), "Xocc", true},
                           {Xact, dbytes(naux * nao * nac), "Xact", true}};
  Plan pl;
  const StepPlan p = plan_step(pl, naux, nao, nocc, nac, np, caller_x);
  const int64_t ncol = nocc + nac;
  if (ncol > 0) {
    if (!check_overlap(c, rs)) return DF_ERR_ARG;
    if (df_status s = need_ws(c, pl.total)) return s;
    rs.push_back({c->ws, pl.total, "workspace", true});
  }
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = enter(c)) return s;
  if (nocc == 0) {
    if (J) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(J, nao * nao, c->stream), "fill");
    if (K) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(K, nao * nao, c->stream), "fill");
    if (v) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(v, naux, c->stream), "fill");
  }
  if (ncol == 0) return DF_OK;
  double* cc = (double*)(c->ws + p.ccat);
  const ColBlock blks[2] = {{Cocc, nocc, nocc, 0}, {Cact, nac, nac, nocc}};
  if (df_status s = pad_operand(c, cc, nao, ncol, blks, 2)) return s;
  double* Xo = caller_x ? Xocc : (double*)(c->ws + p.xo);
  double* Xa = caller_x ? Xact : (double*)(c->ws + p.xa);
  const dfk::OutMap ox = out_split(Xo, Xa, naux, nao, nocc, nac);
  double* vv = nocc > 0 && (J || v) ? (v ? v : (double*)(c->ws + p.vtmp)) : nullptr;
  if (vv)   // v_P from the half transform's epilogue: X_occ is not read again for it
    DF_LAUNCH(DF_KERNEL_HALF_TRANSFORM,
              dfk::launch_half_transform_jvec(B, naux, nao, cc, ncol, ncol, ox, w, nocc, (double*)(c->ws + p.vpart),
                                              vv, 0, c->stream),
              "half transform launch");
  else if (df_status s = run_half(c, B, naux, nao, cc, ncol, ox))
    return s;
  if (nocc > 0) {
    if (J) DF_LAUNCH(DF_KERNEL_COULOMB, dfk::launch_coulomb(B, naux, nao, vv, 1, J, c->stream), "Coulomb launch");
    if (K)
      if (df_status s = run_k(c, Xo, w, naux, nao, nocc, nocc, 1, p.nsplit, (double*)(c->ws + p.kpart), K))
        return s;
  }
  if (nac > 0 && (eri || papa)) {
    double* buv = (double*)(c->ws + p.buv);
    if (df_status s = run_mo(c, Cact, nac, Xa, naux, nao, nac, buv)) return s;
    if (eri)
      if (df_status s = run_pgemm(c, DF_KERNEL_ERI, buv, nac * nac, buv, nac * nac, naux, eri)) return s;
    if (papa && np > 0) {
      double* bpu = (double*)(c->ws + p.bpu);
      if (df_status s = run_mo(c, Cp, np, Xa, naux, nao, nac, bpu)) return s;
      if (df_status s = run_pgemm(c, DF_KERNEL_PAPA, bpu, np * nac, buv, nac * nac, naux, papa)) return s;
    }
  }
  return DF_OK;
}

// dCocc = 2 M Cocc,  M = sum_P <b^P, gJ> b^P  (the Coulomb part of the adjoint, FP64)
static df_status bwd_coulomb(df_ctx* c, char* ws, const BwdPlan& p, const double* B, int64_t naux, int64_t nao,
                             const double* gJ, const double* Cocc, int64_t nocc, double* dCocc) {
  double* g = (double*)(ws + p.g);
  double* u = (double*)(ws + p.u);
  double* M = (double*)(ws + p.M);
  DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_pair_weights(gJ, nao, g, c->stream), "pair weights");
  DF_LAUNCH(DF_KERNEL_JVEC, dfk::launch_jvec_packed(B, naux, nao, g, (double*)(ws + p.upart), u, c->stream),
            "J-vector launch");
  DF_LAUNCH(DF_KERNEL_COULOMB, dfk::launch_coulomb(B, naux, nao, u, 1, M, c->stream), "Coulomb launch");
  const dfk::OpMap A = dfk::op_map(M, nao, nao, nao, 1);
  const dfk::OpMap Bm = dfk::op_map(Cocc, nocc, 1, nao, nocc);
  dfk::OutMap O = dfk::out_plain(dCocc, nao, nocc, nocc);
  O.alpha = 2.0;
  DF_LAUNCH(DF_KERNEL_ADJOINT, dfk::launch_gemm(A, Bm, O, 1, c->stream), "adjoint product");
  return DF_OK;
}

// The active-space part of the adjoint for auxiliary rows [p0, p0 + pc) (FP64):
//   dCact (+)= sum_P X^act_P (Z_P + Z_P^T),  Z_P[uv] = sum_wx Gs[uv][wx] b^P_wx,
// with Gs = geri + geri^T already in ws + p.Gs.  Xa: those rows' X^act, AO-major (rows mu of
// stride ld, columns (P, u) of the chunk).
static df_status bwd_active_rows(df_ctx* c, char* ws, const BwdPlan& p, int64_t pc, int64_t nao, const double* Cact,
                                 int64_t nac, const double* Xa, int64_t ld, double* dCact, int accumulate) {
  const int64_t n2 = nac * nac;
  const double* Gs = (const double*)(ws + p.Gs);
  double* buv = (double*)(ws + p.buv);
  double* Z = (double*)(ws + p.Z);
  if (df_status s = run_mo_ld(c, Cact, nac, Xa, ld, pc, nao, nac, buv)) return s;
  const dfk::OpMap A = dfk::op_map(buv, pc, n2, n2, 1);
  const dfk::OpMap Bm = dfk::op_map(Gs, n2, n2, n2, 1);
  DF_LAUNCH(DF_KERNEL_ADJOINT, dfk::launch_gemm(A, Bm, dfk::out_plain(Z, pc, n2, n2), 1, c->stream),
            "adjoint product");
  DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_symmetrize(Z, nac, pc, Z, c->stream), "symmetrize");
  const dfk::OpMap Ax = dfk::op_map(Xa, nao, ld, pc * nac, 1);
  const dfk::OpMap Bz = dfk::op_map(Z, nac, 1, pc * nac, nac);
  dfk::OutMap O = dfk::out_plain(dCact, nao, nac, nac);
  O.accumulate = accumulate;
  const int nsa = dfk::gemm_splits(nao, nac, (pc * nac + 15) / 16);
  DF_LAUNCH(DF_KERNEL_ADJOINT, dfk::launch_gemm_split(Ax, Bz, O, nsa, (double*)(ws + p.apart), c->stream),
            "adjoint product");
  return DF_OK;
}

// The active-space part of the adjoint over all naux rows at once (Xa AO-major [nao][naux][nac]).
static df_status bwd_active(df_ctx* c, char* ws, const BwdPlan& p, int64_t naux, int64_t nao, const double* Cact,
                            int64_t nac, const double* geri, const double* Xa, double* dCact) {
  DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_symmetrize(geri, nac * nac, 1, (double*)(ws + p.Gs), c->stream), "symmetrize");
  return bwd_active_rows(c, ws, p, naux, nao, Cact, nac, Xa, naux * nac, dCact, 0);
}

df_status df_step_backward(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, const double* Cocc,
                           int64_t nocc, const double* Cact, int64_t nac, const double* gJ, const double* gK,
                           const double* geri, const double* Xocc, const double* Xact, double* dCocc,
                           double* dCact, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (df_status s = check_core(c, B, naux, nao)) return s;
  if (flags != 0) return fail(c, DF_ERR_UNSUPPORTED, "df_step_backward takes no flags");
  if (nocc < 0 || nac < 0) return fail(c, DF_ERR_SHAPE, "sizes must be >= 0");
  if (nocc > 0 && (!Cocc || !dCocc)) return fail(c, DF_ERR_ARG, "Cocc and dCocc are required when nocc > 0");
  if (nac > 0 && (!Cact || !dCact)) return fail(c, DF_ERR_ARG, "Cact and dCact are required when nac > 0");
  const bool caller_x = Xocc != nullptr || Xact != nullptr;
  if (caller_x && ((nocc > 0 && !Xocc) || (nac > 0 && !Xact)))
    return fail(c, DF_ERR_ARG, "Xocc and Xact must be given together (NULL only for an empty one)");
  const int pflags = (gJ ? DF_BWD_GJ : 0) | (gK ? DF_BWD_GK : 0) | (geri ? DF_BWD_GERI : 0) | (caller_x ? DF_CALLER_X : 0);
  const int64_t npair = nao * (nao + 1) / 2;
  std::vector<Range> rs = {{B, dbytes(naux * npair), "B", false},
                           {Cocc, dbytes(nao * nocc), "Cocc", false},
                           {Cact, dbytes(nao * nac), "Cact", false},
                           {gJ, dbytes(nao * nao), "gJ", false},
                           {gK, dbytes(nao * nao), "gK", false},
                           {geri, dbytes(nac * nac * nac * nac), "geri", false},
                           {Xocc, dbytes(naux * nao * nocc), "Xocc", false},
                           {Xact, dbytes(naux * nao * nac), "Xact", false},
                           {dCocc, dbytes(nao * nocc), "dCocc", true},
                           {dCact, dbytes(nao * nac), "dCact", true}};
  const int64_t rows = backward_rows(naux, nao, nocc, nac, pflags, c->scratch_limit);
  if (rows == 0)
    return fail(c, DF_ERR_WORKSPACE, "the scratch limit of " + std::to_string(c->scratch_limit) +
                                         " bytes is below the workspace of one auxiliary row");
  Plan pl;
  const BwdPlan p = plan_backward(pl, naux, nao, nocc, nac, pflags, rows);
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = need_ws(c, pl.total)) return s;
  if (pl.total) rs.push_back({c->ws, pl.total, "workspace", true});
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = enter(c)) return s;
  char* ws = c->ws;
  const bool do_j = gJ && nocc > 0, do_k = gK && nocc > 0, do_e = geri && nac > 0;
  if (nocc > 0 && !do_j && !do_k)
    DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(dCocc, nao * nocc, c->stream), "fill");
  if (nac > 0 && !do_e) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(dCact, nao * nac, c->stream), "fill");
  if (do_j)
    if (df_status s = bwd_coulomb(c, ws, p, B, naux, nao, gJ, Cocc, nocc, dCocc)) return s;
  if (!do_k && !do_e) return DF_OK;
  double* S = (double*)(ws + p.S);
  if (do_k) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_symmetrize(gK, nao, 1, S, c->stream), "symmetrize");
  if (do_e)
    DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_symmetrize(geri, nac * nac, 1, (double*)(ws + p.Gs), c->stream),
              "symmetrize");
  // the forward's half transforms are recomputed, chunk by chunk, when not supplied
  const bool recompute = !caller_x;
  const int64_t no = do_k ? nocc : 0, na = do_e ? nac : 0;
  double* cc = (double*)(ws + p.ccat);
  if (recompute) {
    const ColBlock blks[2] = {{Cocc, nocc, no, 0}, {Cact, nac, na, no}};
    if (df_status s = pad_operand(c, cc, nao, no + na, blks, 2)) return s;
  }
  const int64_t kp = dfk::kpad16(nao);
  // auxiliary rows in chunks of p.chunk; each chunk's share of dCocc and dCact is added in order
  for (int64_t p0 = 0; p0 < naux; p0 += p.chunk) {
    const int64_t pc = std::min(p.chunk, naux - p0);
    const double* Bc = B + p0 * npair;
    const double* Xo;
    const double* Xa;
    int64_t lda;   // row stride of the chunk's AO-major X^act
    if (recompute) {
      double* xo = do_k ? (double*)(ws + p.xo) : nullptr;
      double* xa = do_e ? (double*)(ws + p.xa) : nullptr;
      if (df_status s = run_half(c, Bc, pc, nao, cc, no + na, out_split(xo, xa, pc, nao, no, na))) return s;
      Xo = xo;
      Xa = xa;
      lda = pc * nac;
    } else {
      Xo = Xocc ? Xocc + p0 * nao * nocc : nullptr;
      Xa = Xact ? Xact + p0 * nac : nullptr;
      lda = naux * nac;
    }
    if (do_k) {
      // dCocc += sum_P b^P Y_P,  Y_P = S X_P,  S = gK + gK^T
      double* Y = (double*)(ws + p.Y);
      const dfk::OpMap A = dfk::op_map(S, nao, nao, nao, 1);
      dfk::OpMap Bm = dfk::op_map(Xo, pc * nocc, 1, nao, nocc);
      Bm.rl = nocc;
      Bm.s_rh = nao * nocc;
      // Y [P][kpad16(nao)][nocc]: the packed product reads whole 16-row slabs of each Y_P
      dfk::OutMap O = dfk::out_plain(Y, nao, pc * nocc, nocc);
      O.nl = nocc;
      O.s_nh = kp * nocc;
      DF_LAUNCH(DF_KERNEL_ADJOINT, dfk::launch_gemm(A, Bm, O, 1, c->stream), "adjoint product");
      if (kp > nao)
        DF_LAUNCH(DF_KERNEL_OTHER,
                  dfk::launch_fill_zero_strided(Y + nao * nocc, pc, kp * nocc, (kp - nao) * nocc, c->stream), "fill");
      dfk::OpMap Ym = dfk::op_map(Y, nocc, 1, nao, nocc);
      Ym.kb_n = pc;
      Ym.s_kb = kp * nocc;
      dfk::OutMap Od = dfk::out_plain(dCocc, nao, nocc, nocc);
      Od.accumulate = do_j || p0 > 0 ? 1 : 0;
      DF_LAUNCH(DF_KERNEL_ADJOINT, dfk::launch_half_reduce(Bc, pc, nao, Ym, Od, (double*)(ws + p.kpart), c->stream),
                "adjoint packed product");
    }
    if (do_e)
      if (df_status s = bwd_active_rows(c, ws, p, pc, nao, Cact, nac, Xa, lda, dCact, p0 > 0)) return s;
  }
  return DF_OK;
}

df_status df_split_matmul(df_ctx* ctx, const double* A, int64_t lda, int64_t M, const double* Bm, int64_t ldb,
                          int64_t N, int64_t K, int nslice, double* C, int64_t ldc, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (flags != 0) return fail(c, DF_ERR_UNSUPPORTED, "df_split_matmul takes no flags");
  if (nslice < 4 || nslice > 8) return fail(c, DF_ERR_SHAPE, "nslice must be in [4, 8]");
  if (M < 0 || N < 0 || K < 1) return fail(c, DF_ERR_SHAPE, "M, N must be >= 0 and K >= 1");
  if (M > 0 && (!A || lda < K)) return fail(c, DF_ERR_ARG, "A is NULL or lda < K");
  if (N > 0 && (!Bm || ldb < K)) return fail(c, DF_ERR_ARG, "B is NULL or ldb < K");
  if (M > 0 && N > 0 && (!C || ldc < N)) return fail(c, DF_ERR_ARG, "C is NULL or ldc < N");
  if (dfk::rpad32(M) > 0x7fffffffLL || dfk::rpad32(N) > 0x7fffffffLL || K > (1LL << 30))
    return fail(c, DF_ERR_SHAPE, "M and N must be below 2^31 - 32 and K at most 2^30");
  std::vector<Range> rs = {{A, dbytes(M > 0 ? (M - 1) * lda + K : 0), "A", false},
                           {Bm, dbytes(N > 0 ? (N - 1) * ldb + K : 0), "B", false},
                           {C, dbytes(M > 0 && N > 0 ? (M - 1) * ldc + N : 0), "C", true}};
  Plan pl;
  const SplitMmPlan p = plan_split_mm(pl, M, N, K, nslice);
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (M == 0 || N == 0) return DF_OK;
  if (df_status s = need_ws(c, pl.total)) return s;
  rs.push_back({c->ws, pl.total, "workspace", true});
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = enter(c)) return s;
  int8_t* ap = (int8_t*)(c->ws + p.a.planes);
  int8_t* bp = (int8_t*)(c->ws + p.b.planes);
  int* ea = (int*)(c->ws + p.a.ex);
  int* eb = (int*)(c->ws + p.b.ex);
  DF_LAUNCH(DF_KERNEL_SPLIT, dfk::launch_split_rows(dfk::op_map(A, M, lda, K, 1), K, nslice, ap, ea, c->stream),
            "split launch");
  DF_LAUNCH(DF_KERNEL_SPLIT, dfk::launch_split_rows(dfk::op_map(Bm, N, ldb, K, 1), K, nslice, bp, eb, c->stream),
            "split launch");
  const dfk::OutMap O = dfk::out_plain(C, M, N, ldc);
  double* part = p.nsplit > 1 ? (double*)(c->ws + p.part) : nullptr;
  DF_LAUNCH(DF_KERNEL_OTHER,
            dfk::launch_slice_gemm(ap, ea, M, bp, eb, N, dfk::kpad64(K), nslice, O, false, p.nsplit, part, c->stream),
            "slice product launch");
  if (part) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_split_reduce(part, p.nsplit, O, c->stream), "split reduce");
  return DF_OK;
}

df_status df_split_cholesky(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, int nslice, int8_t* Bs,
                            int* Be, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (df_status s = check_core(c, B, naux, nao)) return s;
  if (flags != 0) return fail(c, DF_ERR_UNSUPPORTED, "df_split_cholesky takes no flags");
  if (nslice < 4 || nslice > 8) return fail(c, DF_ERR_SHAPE, "nslice must be in [4, 8]");
  if (!Bs || !Be) return fail(c, DF_ERR_ARG, "Bs and Be are required");
  if ((uintptr_t)Bs % 16 != 0) return fail(c, DF_ERR_ARG, "Bs must be 16-byte aligned");
  if (dfk::rpad32(naux * nao) > 0x7fffffffLL) return fail(c, DF_ERR_SHAPE, "naux * nao must be below 2^31 - 32");
  const int64_t npair = nao * (nao + 1) / 2;
  std::vector<Range> rs = {{B, dbytes(naux * npair), "B", false},
                           {Bs, (size_t)dfk::split_plane_bytes(naux * nao, nao, nslice), "Bs", true},
                           {Be, (size_t)naux * nao * 4, "Be", true}};
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = enter(c)) return s;
  DF_LAUNCH(DF_KERNEL_SPLIT, dfk::launch_split_packed(B, naux, nao, nslice, Bs, Be, c->stream), "split launch");
  return DF_OK;
}

df_status df_step_split(df_ctx* ctx, const double* B, const int8_t* Bs, const int* Be, int nslice, int64_t naux,
                        int64_t nao, const double* Cocc, int64_t nocc, const double* Cact, int64_t nac,
                        const double* Cp, int64_t np, double* J, double* K, double* v, double* eri, double* papa,
                        double* Xocc, double* Xact, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (df_status s = check_core(c, B, naux, nao)) return s;
  if (flags != 0) return fail(c, DF_ERR_UNSUPPORTED, "df_step_split takes no flags");
  const bool caller_x = Xocc != nullptr || Xact != nullptr;
  if (caller_x && ((nocc > 0 && !Xocc) || (nac > 0 && !Xact)))
    return fail(c, DF_ERR_ARG, "Xocc and Xact must be given together (NULL only for an empty one)");
  if (nslice < 4 || nslice > 8) return fail(c, DF_ERR_SHAPE, "nslice must be in [4, 8]");
  if (!Bs || !Be) return fail(c, DF_ERR_ARG, "Bs and Be (from df_split_cholesky) are required");
  if ((uintptr_t)Bs % 16 != 0) return fail(c, DF_ERR_ARG, "Bs must be 16-byte aligned");
  if (nocc < 0 || nac < 0 || np < 0) return fail(c, DF_ERR_SHAPE, "sizes must be >= 0");
  if (nocc > 0 && !Cocc) return fail(c, DF_ERR_ARG, "Cocc is NULL");
  if (nac > 0 && !Cact) return fail(c, DF_ERR_ARG, "Cact is NULL");
  if (np > 0 && !Cp) return fail(c, DF_ERR_ARG, "Cp is NULL");
  if (dfk::rpad32(naux * nao) > 0x7fffffffLL || dfk::rpad32(naux * nac) > 0x7fffffffLL ||
      dfk::rpad32(np * nac) > 0x7fffffffLL || naux * nocc > (1LL << 30))
    return fail(c, DF_ERR_SHAPE, "problem too large for the split path");
  const int64_t npair = nao * (nao + 1) / 2;
  const int64_t ncol = nocc + nac;
  std::vector<Range> rs = {{B, dbytes(naux * npair), "B", false},
                           {Bs, (size_t)dfk::split_plane_bytes(naux * nao, nao, nslice), "Bs", false},
                           {Be, (size_t)naux * nao * 4, "Be", false},
                           {Cocc, dbytes(nao * nocc), "Cocc", false},
                           {Cact, dbytes(nao * nac), "Cact", false},
                           {Cp, dbytes(nao * np), "Cp", false},
                           {J, dbytes(nao * nao), "J", true},
                           {K, dbytes(nao * nao), "K", true},
                           {v, dbytes(naux), "v", true},
                           {eri, dbytes(nac * nac * nac * nac), "eri", true},
                           {papa, dbytes(np * nac * nac * nac), "papa", true},
                           {Xocc, dbytes(naux * nao * nocc), "Xocc", true},
                           {Xact, dbytes(naux * nao * nac), "Xact", true}};
  Plan pl;
  const StepSplitPlan p = plan_step_split(pl, naux, nao, nocc, nac, np, nslice, caller_x);
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = need_ws(c, pl.total)) return s;
  rs.push_back({c->ws, pl.total, "workspace", true});
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = enter(c)) return s;
  char* ws = c->ws;
  if (nocc == 0) {
    if (J) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(J, nao * nao, c->stream), "fill");
    if (K) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(K, nao * nao, c->stream), "fill");
    if (v) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(v, naux, c->stream), "fill");
  }
  if (ncol == 0) return DF_OK;
  const int64_t kpo = dfk::kpad64(nao);
  // a2: X[(P, m)][c] = sum_k b^P_{mk} [Cact | Cocc][k][c], against the pre-split rows of b^P;
  // X_act goes out AO-major [m][P][u], X_occ P-major [P][m][i] (the layouts of df_step)
  double* cc = (double*)(ws + p.ccat);
  const ColBlock blks[2] = {{Cact, nac, nac, 0}, {Cocc, nocc, nocc, nac}};
  if (df_status s = pad_operand_plain(c, cc, nao, ncol, blks, 2)) return s;
  int8_t* cs = (int8_t*)(ws + p.cs.planes);
  int* ce = (int*)(ws + p.cs.ex);
  DF_LAUNCH(DF_KERNEL_SPLIT, dfk::launch_split_rows(dfk::op_map(cc, ncol, 1, nao, ncol), nao, nslice, cs, ce, c->stream),
            "split launch");
  double* Xo = caller_x ? Xocc : (double*)(ws + p.xo);
  double* Xa = caller_x ? Xact : (double*)(ws + p.xa);
  dfk::OutMap OX = dfk::out_plain(Xa, naux * nao, ncol, naux * nac);
  OX.ml = nao;       // m = (P, mu): P * nac + mu * naux * nac
  OX.s_mh = nac;
  OX.nsplit = nac;
  OX.p2 = Xo;
  OX.s2_m = nocc;
  DF_LAUNCH(DF_KERNEL_HALF_TRANSFORM,
            dfk::launch_slice_gemm(Bs, Be, naux * nao, cs, ce, ncol, kpo, nslice, OX, false, 1, nullptr, c->stream),
            "slice product launch");
  if (nocc > 0) {
    // a3, a4 in FP64
    if (J || v) {
      double* vv = v ? v : (double*)(ws + p.vtmp);
      DF_LAUNCH(DF_KERNEL_JVEC, dfk::launch_jvec(Xo, naux, nao, nocc, Cocc, nullptr, nocc, 1, vv, c->stream),
                "J-vector launch");
      if (J) DF_LAUNCH(DF_KERNEL_COULOMB, dfk::launch_coulomb(B, naux, nao, vv, 1, J, c->stream), "Coulomb launch");
    }
    // a5: K = sum_{P, c} X[P][i][c] X[P][j][c] from the split rows i of X_occ
    if (K) {
      dfk::OpMap ox = dfk::op_map(Xo, nao, nocc, nocc, 1);
      ox.kb_n = naux;
      ox.s_kb = nao * nocc;
      int8_t* xs = (int8_t*)(ws + p.xos.planes);
      int* xe = (int*)(ws + p.xos.ex);
      DF_LAUNCH(DF_KERNEL_SPLIT, dfk::launch_split_rows(ox, naux * nocc, nslice, xs, xe, c->stream), "split launch");
      double* kpart = (double*)(ws + p.kpart);
      const dfk::OutMap OK = dfk::out_plain(kpart, nao, nao, nao);
      DF_LAUNCH(DF_KERNEL_K_SYRK,
                dfk::launch_slice_gemm(xs, xe, nao, xs, xe, nao, dfk::kpad64(naux * nocc), nslice, OK, true, p.nsk,
                                       p.nsk > 1 ? kpart : nullptr, c->stream),
                "slice product launch");
      DF_LAUNCH(DF_KERNEL_K_REDUCE, dfk::launch_syrk_reduce(kpart, p.nsk, nao, 1, K, c->stream), "K reduce launch");
    }
  }
  if (nac > 0 && (eri || papa)) {
    // a6: b^P_{pu} = sum_mu Cp[mu][p] X[mu][P][u]; split rows (P, u) of X_act and rows p of Cp
    const dfk::OpMap oxa = dfk::op_map(Xa, naux * nac, 1, nao, naux * nac);
    int8_t* xas = (int8_t*)(ws + p.xas.planes);
    int* xae = (int*)(ws + p.xas.ex);
    DF_LAUNCH(DF_KERNEL_SPLIT, dfk::launch_split_rows(oxa, nao, nslice, xas, xae, c->stream), "split launch");
    auto second = [&](const double* Cl, int64_t nl, const SplitBuf& sb, double* out) -> df_status {
      int8_t* ls = (int8_t*)(ws + sb.planes);
      int* le = (int*)(ws + sb.ex);
      DF_LAUNCH(DF_KERNEL_SPLIT, dfk::launch_split_rows(dfk::op_map(Cl, nl, 1, nao, nl), nao, nslice, ls, le, c->stream),
                "split launch");
      dfk::OutMap O = dfk::out_plain(out, nl, naux * nac, nac);
      O.nl = nac;
      O.s_nh = nl * nac;
      DF_LAUNCH(DF_KERNEL_MO_TRANSFORM,
                dfk::launch_slice_gemm(ls, le, nl, xas, xae, naux * nac, kpo, nslice, O, false, 1, nullptr, c->stream),
                "slice product launch");
      return DF_OK;
    };
    double* buv = (double*)(ws + p.buv);
    if (df_status s = second(Cact, nac, p.cas, buv)) return s;
    const int64_t n2 = nac * nac;
    int8_t* bvs = (int8_t*)(ws + p.buvs.planes);
    int* bve = (int*)(ws + p.buvs.ex);
    DF_LAUNCH(DF_KERNEL_SPLIT, dfk::launch_split_rows(dfk::op_map(buv, n2, 1, naux, n2), naux, nslice, bvs, bve, c->stream),
              "split launch");
    const int64_t kpa = dfk::kpad64(naux);
    // a8: (uv|wx) = sum_P b^P_uv b^P_wx
    if (eri)
      DF_LAUNCH(DF_KERNEL_ERI,
                dfk::launch_slice_gemm(bvs, bve, n2, bvs, bve, n2, kpa, nslice, dfk::out_plain(eri, n2, n2, n2), false,
                                       1, nullptr, c->stream),
                "slice product launch");
    // a7: (pu|vw) = sum_P b^P_pu b^P_vw
    if (papa && np > 0) {
      double* bpu = (double*)(ws + p.bpu);
      if (df_status s = second(Cp, np, p.cps, bpu)) return s;
      int8_t* bps = (int8_t*)(ws + p.bpus.planes);
      int* bpe = (int*)(ws + p.bpus.ex);
      DF_LAUNCH(DF_KERNEL_SPLIT,
                dfk::launch_split_rows(dfk::op_map(bpu, np * nac, 1, naux, np * nac), naux, nslice, bps, bpe, c->stream),
                "split launch");
      DF_LAUNCH(DF_KERNEL_PAPA,
                dfk::launch_slice_gemm(bps, bpe, np * nac, bvs, bve, n2, kpa, nslice, dfk::out_plain(papa, np * nac, n2, n2),
                                       false, 1, nullptr, c->stream),
                "slice product launch");
    }
  }
  return DF_OK;
}

df_status df_set_autotune(df_ctx* ctx, int enable) {
  if (!ctx) return DF_ERR_ARG;
  ctx->autotune = enable != 0;
  return DF_OK;
}

df_status df_batched_tuning(df_ctx* ctx, const df_problem* probs, int nprob, int* half_tile_n, int* k_tile,
                            int* k_rounds, int* tuned) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (nprob < 0 || (nprob > 0 && !probs)) return fail(c, DF_ERR_ARG, "probs is NULL");
  if (!half_tile_n || !k_tile || !k_rounds || !tuned) return fail(c, DF_ERR_ARG, "output pointers are NULL");
  BatchedTune tu = batched_default_tune(probs, nprob);
  resolve_arch(c);
  const BatchedTune* known = tune_find(c, batched_key(probs, nprob));
  *tuned = known != nullptr;
  if (known) tu = *known;
  *half_tile_n = tu.half_n;
  *k_tile = tu.k_tile;
  *k_rounds = tu.k_rounds;
  return DF_OK;
}

df_status df_batched_set_tuning(df_ctx* ctx, const df_problem* probs, int nprob, int half_tile_n, int k_tile,
                                int k_rounds) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (nprob < 0 || (nprob > 0 && !probs)) return fail(c, DF_ERR_ARG, "probs is NULL");
  const BatchedTune t{half_tile_n, k_tile, k_rounds};
  if (!tune_valid(t)) return fail(c, DF_ERR_ARG, "not a candidate configuration");
  const std::string shape = batched_key(probs, nprob);
  resolve_arch(c);
  if (!c->arch.empty()) c->tune.erase(c->arch + "|" + shape);   // the stored choice is this one
  c->tune["|" + shape] = t;
  return DF_OK;
}

df_status df_autotune_save(df_ctx* ctx, const char* path) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (!path || !*path) return fail(c, DF_ERR_ARG, "path is empty");
  std::string err;
  if (!tune_write(c, path, &err)) return fail(c, DF_ERR_ARG, err);
  return DF_OK;
}

df_status df_autotune_load(df_ctx* ctx, const char* path) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (!path || !*path) return fail(c, DF_ERR_ARG, "path is empty");
  std::string err;
  if (!tune_read(c, path, &err)) return fail(c, DF_ERR_ARG, err);
  return DF_OK;
}

df_status df_split_cholesky_t(df_ctx* ctx, const double* B, int64_t naux, int64_t nao, int nslice, int8_t* Bt,
                              int* Bte, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (df_status s = check_core(c, B, naux, nao)) return s;
  if (flags != 0) return fail(c, DF_ERR_UNSUPPORTED, "df_split_cholesky_t takes no flags");
  if (nslice < 4 || nslice > 8) return fail(c, DF_ERR_SHAPE, "nslice must be in [4, 8]");
  if (!Bt || !Bte) return fail(c, DF_ERR_ARG, "Bt and Bte are required");
  if ((uintptr_t)Bt % 16 != 0) return fail(c, DF_ERR_ARG, "Bt must be 16-byte aligned");
  if (naux * nao > (1LL << 30)) return fail(c, DF_ERR_SHAPE, "naux * nao must be at most 2^30");
  const int64_t npair = nao * (nao + 1) / 2;
  std::vector<Range> rs = {{B, dbytes(naux * npair), "B", false},
                           {Bt, (size_t)dfk::split_plane_bytes(nao, naux * nao, nslice), "Bt", true},
                           {Bte, (size_t)nao * 4, "Bte", true}};
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = enter(c)) return s;
  DF_LAUNCH(DF_KERNEL_SPLIT, dfk::launch_split_packed_t(B, naux, nao, nslice, Bt, Bte, c->stream), "split launch");
  return DF_OK;
}

df_status df_step_backward_split(df_ctx* ctx, const double* B, const int8_t* Bt, const int* Bte, int nslice,
                                 int64_t naux, int64_t nao, const double* Cocc, int64_t nocc, const double* Cact,
                                 int64_t nac, const double* gJ, const double* gK, const double* geri,
                                 const double* Xocc, const double* Xact, double* dCocc, double* dCact, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (df_status s = check_core(c, B, naux, nao)) return s;
  if (flags != 0) return fail(c, DF_ERR_UNSUPPORTED, "df_step_backward_split takes no flags");
  if (nslice < 4 || nslice > 8) return fail(c, DF_ERR_SHAPE, "nslice must be in [4, 8]");
  if (nocc < 0 || nac < 0) return fail(c, DF_ERR_SHAPE, "sizes must be >= 0");
  if (nocc > 0 && (!Cocc || !dCocc)) return fail(c, DF_ERR_ARG, "Cocc and dCocc are required when nocc > 0");
  if (nac > 0 && (!Cact || !dCact)) return fail(c, DF_ERR_ARG, "Cact and dCact are required when nac > 0");
  const bool do_j = gJ && nocc > 0, do_k = gK && nocc > 0, do_e = geri && nac > 0;
  if (do_k && (!Xocc || !Bt || !Bte)) return fail(c, DF_ERR_ARG, "gK needs Xocc and Bt, Bte (df_split_cholesky_t)");
  if (do_e && !Xact) return fail(c, DF_ERR_ARG, "geri needs Xact");
  if (Bt && (uintptr_t)Bt % 16 != 0) return fail(c, DF_ERR_ARG, "Bt must be 16-byte aligned");
  if (nao > 32768 || naux * nao > (1LL << 30) || dfk::rpad32(naux * nocc) > 0x7fffffffLL)
    return fail(c, DF_ERR_SHAPE, "problem too large for the split path");
  const int pflags = (gJ ? DF_BWD_GJ : 0) | (gK ? DF_BWD_GK : 0) | (geri ? DF_BWD_GERI : 0);
  const int64_t npair = nao * (nao + 1) / 2;
  std::vector<Range> rs = {{B, dbytes(naux * npair), "B", false},
                           {Bt, (size_t)dfk::split_plane_bytes(nao, naux * nao, nslice), "Bt", false},
                           {Bte, (size_t)nao * 4, "Bte", false},
                           {Cocc, dbytes(nao * nocc), "Cocc", false},
                           {Cact, dbytes(nao * nac), "Cact", false},
                           {gJ, dbytes(nao * nao), "gJ", false},
                           {gK, dbytes(nao * nao), "gK", false},
                           {geri, dbytes(nac * nac * nac * nac), "geri", false},
                           {Xocc, dbytes(naux * nao * nocc), "Xocc", false},
                           {Xact, dbytes(naux * nao * nac), "Xact", false},
                           {dCocc, dbytes(nao * nocc), "dCocc", true},
                           {dCact, dbytes(nao * nac), "dCact", true}};
  Plan pl;
  const BwdSplitPlan p = plan_backward_split(pl, naux, nao, nocc, nac, pflags, nslice);
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = need_ws(c, pl.total)) return s;
  if (pl.total) rs.push_back({c->ws, pl.total, "workspace", true});
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = enter(c)) return s;
  char* ws = c->ws;
  if (nocc > 0 && !do_j && !do_k) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(dCocc, nao * nocc, c->stream), "fill");
  if (nac > 0 && !do_e) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(dCact, nao * nac, c->stream), "fill");
  if (do_j)
    if (df_status s = bwd_coulomb(c, ws, p.f, B, naux, nao, gJ, Cocc, nocc, dCocc)) return s;
  if (do_k) {
    // dCocc += sum_P b^P Y_P,  Y_P = S X_P,  S = gK + gK^T.  Y_P in FP64 (the tall product of
    // the FP64 adjoint: it takes about what the slice product takes, and needs no split of S and
    // X), the sum over (P, nu) from int8 slices of B and Y
    double* S = (double*)(ws + p.S);
    double* Y = (double*)(ws + p.Y);
    DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_symmetrize(gK, nao, 1, S, c->stream), "symmetrize");
    const int64_t kpb = dfk::kpad64(naux * nao);
    int8_t* ys = (int8_t*)(ws + p.ys.planes);
    int* ye = (int*)(ws + p.ys.ex);
    // Y[P][mu][i] = sum_nu S[mu][nu] X[P][nu][i]
    dfk::OpMap Xm = dfk::op_map(Xocc, naux * nocc, 1, nao, nocc);
    Xm.rl = nocc;
    Xm.s_rh = nao * nocc;
    dfk::OutMap OY = dfk::out_plain(Y, nao, naux * nocc, nocc);
    OY.nl = nocc;
    OY.s_nh = nao * nocc;
    DF_LAUNCH(DF_KERNEL_ADJOINT, dfk::launch_gemm(dfk::op_map(S, nao, nao, nao, 1), Xm, OY, 1, c->stream),
              "adjoint product");
    // rows i of Y over (P, nu); then dCocc[mu][i] += sum_{P, nu} b^P_{mu nu} Y[P][nu][i]
    dfk::OpMap oy = dfk::op_map(Y, nocc, 1, nao, nocc);
    oy.kb_n = naux;
    oy.s_kb = nao * nocc;
    DF_LAUNCH(DF_KERNEL_SPLIT, dfk::launch_split_rows(oy, naux * nao, nslice, ys, ye, c->stream), "split launch");
    dfk::OutMap Od = dfk::out_plain(dCocc, nao, nocc, nocc);
    Od.accumulate = do_j ? 1 : 0;
    double* part = p.nsk > 1 ? (double*)(ws + p.part) : nullptr;
    DF_LAUNCH(DF_KERNEL_ADJOINT,
              dfk::launch_slice_gemm(Bt, Bte, nao, ys, ye, nocc, kpb, nslice, Od, false, p.nsk, part, c->stream),
              "slice product launch");
    if (part) DF_LAUNCH(DF_KERNEL_ADJOINT, dfk::launch_split_reduce(part, p.nsk, Od, c->stream), "split reduce");
  }
  if (do_e)
    if (df_status s = bwd_active(c, ws, p.f, naux, nao, Cact, nac, geri, Xact, dCact)) return s;
  return DF_OK;
}

df_status df_batched_workspace_size(const df_problem* probs, int nprob, size_t* bytes) {
  if (!bytes || nprob < 0 || (nprob > 0 && !probs)) return DF_ERR_ARG;
  *bytes = 0;
  for (int i = 0; i < nprob; ++i) {
    const df_problem& q = probs[i];
    if (q.naux < 1 || q.nao < 1 || q.nao > kMaxNao || q.ndm < 1 || q.nocc < 0 || q.nac < 0 || q.np < 0)
      return DF_ERR_SHAPE;
  }
  Plan pl;
  plan_batched(pl, probs, nprob);
  *bytes = pl.total + batched_ppaa_bytes(probs, nprob);
  return DF_OK;
}

// J (FP64) of problem q from its J-vectors: V B^T over the packed pairs for many densities, else
// the Coulomb kernel.  v comes from X_occ (Xo) or, when that is the larger read, from packed B.
static df_status batched_coulomb(df_ctx* c, const df_problem& q, const double* Xo, double* v, double* jp,
                                 double* dfull, double* dw, int vsplit, double* vpart) {
  const int64_t npair = q.nao * (q.nao + 1) / 2;
  if (batched_jvec_from_b(q)) {
    DF_LAUNCH(DF_KERNEL_JVEC, dfk::launch_dens_pairs(q.Cocc, q.nao, q.nocc, q.ndm, dfull, dw, c->stream),
              "density launch");
    const dfk::OpMap A = dfk::op_map(dw, q.ndm, npair, npair, 1);
    const dfk::OpMap Bm = dfk::op_map(q.B, q.naux, npair, npair, 1);
    DF_LAUNCH(DF_KERNEL_JVEC,
              dfk::launch_gemm_split(A, Bm, dfk::out_plain(v, q.ndm, q.naux, q.naux), vsplit, vpart, c->stream),
              "J-vector product launch");
  } else {
    DF_LAUNCH(DF_KERNEL_JVEC,
              dfk::launch_jvec(Xo, q.naux, q.nao, q.ndm * q.nocc, q.Cocc, nullptr, q.nocc, q.ndm, v, c->stream),
              "J-vector launch");
  }
  if (batched_j_gemm(q)) {
    const dfk::OpMap A = dfk::op_map(v, q.ndm, q.naux, q.naux, 1);
    const dfk::OpMap Bm = dfk::op_map(q.B, npair, 1, q.naux, npair);
    DF_LAUNCH(DF_KERNEL_COULOMB, dfk::launch_gemm(A, Bm, dfk::out_plain(jp, q.ndm, npair, npair), 1, c->stream),
              "Coulomb product launch");
    DF_LAUNCH(DF_KERNEL_COULOMB, dfk::launch_unpack_sym(jp, q.ndm, q.nao, q.J, c->stream), "unpack launch");
  } else {
    DF_LAUNCH(DF_KERNEL_COULOMB, dfk::launch_coulomb(q.B, q.naux, q.nao, v, q.ndm, q.J, c->stream), "Coulomb launch");
  }
  return DF_OK;
}

df_status df_batched_step(df_ctx* ctx, const df_problem* probs, int nprob, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (flags != 0) return fail(c, DF_ERR_UNSUPPORTED, "df_batched_step takes no flags");
  if (nprob < 0 || (nprob > 0 && !probs)) return fail(c, DF_ERR_ARG, "probs is NULL");
  std::vector<Range> rs;
  for (int i = 0; i < nprob; ++i) {
    const df_problem& q = probs[i];
    const std::string tag = "problem " + std::to_string(i) + " ";
    if (df_status s = check_core(c, q.B, q.naux, q.nao)) return s;
    if (q.ndm < 1 || q.ndm > 65535 || q.nocc < 0 || q.nac < 0 || q.np < 0)
      return fail(c, DF_ERR_SHAPE, tag + "has a bad size");
    if (q.nocc > 0 && (q.J || q.K) && !q.Cocc) return fail(c, DF_ERR_ARG, tag + "Cocc is NULL");
    if (q.nac > 0 && (q.eri || q.papa) && !q.Cact) return fail(c, DF_ERR_ARG, tag + "Cact is NULL");
    if (q.np > 0 && q.papa && !q.Cp) return fail(c, DF_ERR_ARG, tag + "Cp is NULL");
    if (wants_ppaa(q) && (!q.Cact || !q.Cp)) return fail(c, DF_ERR_ARG, tag + "ppaa needs Cact and Cp");
    const int64_t npair = q.nao * (q.nao + 1) / 2;
    rs.push_back({q.B, dbytes(q.naux * npair), "B", false});
    rs.push_back({q.ppaa, dbytes(q.nac * (q.nac + 1) / 2 * q.np * q.np), "ppaa", true});
    rs.push_back({q.Cocc, dbytes(q.ndm * q.nao * q.nocc), "Cocc", false});
    rs.push_back({q.Cact, dbytes(q.nao * q.nac), "Cact", false});
    rs.push_back({q.Cp, dbytes(q.nao * q.np), "Cp", false});
    rs.push_back({q.J, dbytes(q.ndm * q.nao * q.nao), "J", true});
    rs.push_back({q.K, dbytes(q.ndm * q.nao * q.nao), "K", true});
    rs.push_back({q.eri, dbytes(q.nac * q.nac * q.nac * q.nac), "eri", true});
    rs.push_back({q.papa, dbytes(q.np * q.nac * q.np * q.nac), "papa", true});
  }
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  Plan pl;
  const std::vector<BatchedPiece> pc = plan_batched(pl, probs, nprob);
  const size_t ppaa_off = pl.total;
  pl.total += batched_ppaa_bytes(probs, nprob);
  if (df_status s = need_ws(c, pl.total)) return s;
  if (pl.total) rs.push_back({c->ws, pl.total, "workspace", true});
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (nprob == 0) return DF_OK;
  if (df_status s = enter(c)) return s;
  char* ws = c->ws;
  // largest first
  std::vector<int> order((size_t)nprob);
  for (int i = 0; i < nprob; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return batched_work(probs[a]) > batched_work(probs[b]); });
  // zero outputs of problems without occupied columns
  for (int i : order) {
    const df_problem& q = probs[i];
    if (q.nocc == 0) {
      if (q.J) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(q.J, q.ndm * q.nao * q.nao, c->stream), "fill");
      if (q.K) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(q.K, q.ndm * q.nao * q.nao, c->stream), "fill");
    }
  }
  // padded operands [C_1 .. C_ndm | Cact] and the descriptors of the grouped half transforms
  std::vector<dfk::GroupHalf> gh;
  for (int i : order) {
    const df_problem& q = probs[i];
    const BatchedPiece& b = pc[(size_t)i];
    const int64_t ncol = batched_ncol(q);
    if (ncol == 0 || !(q.J || q.K || q.eri || q.papa)) continue;
    double* cp = (double*)(ws + b.cpad);
    std::vector<ColBlock> blks;
    for (int64_t z = 0; z < q.ndm; ++z) blks.push_back({q.Cocc + z * q.nao * q.nocc, q.nocc, q.nocc, z * q.nocc});
    blks.push_back({q.Cact, q.nac, q.nac, q.ndm * q.nocc});
    if (df_status s = pad_operand(c, cp, q.nao, ncol, blks.data(), (int)blks.size())) return s;
    double* Xo = (double*)(ws + b.xo);
    double* Xa = (double*)(ws + b.xa);
    gh.push_back({q.B, q.naux, q.nao, cp, ncol, ncol, out_split(Xo, Xa, q.naux, q.nao, q.ndm * q.nocc, q.nac)});
  }
  auto run_half = [&](int tile_n) -> df_status {
    for (size_t g0 = 0; g0 < gh.size(); g0 += dfk::kMaxGroup) {
      const int n = (int)std::min<size_t>(dfk::kMaxGroup, gh.size() - g0);
      DF_LAUNCH(DF_KERNEL_HALF_TRANSFORM, dfk::launch_half_group(gh.data() + g0, n, tile_n, c->stream),
                "grouped half transform");
    }
    return DF_OK;
  };
  // grouped K tiles with the split counts of (tile, rounds), then the fixed-order reductions
  auto run_k = [&](int tile, int rounds) -> df_status {
    const std::vector<int> ns = batched_k_splits(probs, nprob, tile, rounds);
    std::vector<dfk::GroupSyrk> gs;
    for (int i : order) {
      const df_problem& q = probs[i];
      if (!q.K || q.nocc <= 0) continue;
      const int64_t no = q.ndm * q.nocc;
      dfk::OpMap A = dfk::op_map((const double*)(ws + pc[(size_t)i].xo), q.nao, no, q.nocc, 1);
      A.kb_n = q.naux;
      A.s_kb = q.nao * no;
      A.s_z = q.nocc;
      gs.push_back({A, q.nao, q.ndm, ns[(size_t)i], (double*)(ws + pc[(size_t)i].kpart)});
    }
    for (size_t g0 = 0; g0 < gs.size(); g0 += dfk::kMaxGroup) {
      const int n = (int)std::min<size_t>(dfk::kMaxGroup, gs.size() - g0);
      DF_LAUNCH(DF_KERNEL_K_SYRK, dfk::launch_syrk_group(gs.data() + g0, n, tile, c->stream), "grouped K tiles");
    }
    for (int i : order) {
      const df_problem& q = probs[i];
      if (!q.K || q.nocc <= 0) continue;
      DF_LAUNCH(DF_KERNEL_K_REDUCE,
                dfk::launch_syrk_reduce((double*)(ws + pc[(size_t)i].kpart), ns[(size_t)i], q.nao, q.ndm, q.K,
                                        c->stream),
                "K reduce launch");
    }
    return DF_OK;
  };
  BatchedTune tu = batched_default_tune(probs, nprob);
  const std::string key = batched_key(probs, nprob);
  resolve_arch(c);
  if (const BatchedTune* known = tune_find(c, key)) {
    tu = *known;
  } else if (c->autotune) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    DF_HIP(hipStreamIsCapturing(c->stream, &cs), "hipStreamIsCapturing");
    if (cs == hipStreamCaptureStatusNone) {
      // time every candidate of each phase twice on these buffers (the best of the two counts);
      // the half transform runs first, so that the K candidates read its X
      hipEvent_t ea = nullptr, eb = nullptr;
      if (df_status s = take_event(c, &ea)) return s;
      if (df_status s = take_event(c, &eb)) {
        c->ev_pool.push_back(ea);
        return s;
      }
      const bool timing = c->timing;
      c->timing = false;
      auto best_of = [&](const auto& run, float* ms) -> df_status {
        *ms = 3.0e38f;
        for (int rep = 0; rep < 2; ++rep) {
          DF_HIP(hipEventRecord(ea, c->stream), "hipEventRecord");
          if (df_status s = run()) return s;
          DF_HIP(hipEventRecord(eb, c->stream), "hipEventRecord");
          DF_HIP(hipEventSynchronize(eb), "hipEventSynchronize");
          float el = 0.0f;
          DF_HIP(hipEventElapsedTime(&el, ea, eb), "hipEventElapsedTime");
          *ms = std::min(*ms, el);
        }
        return DF_OK;
      };
      auto tune_all = [&]() -> df_status {
        float best = 3.0e38f, ms = 0.0f;
        for (int tn : kHalfTiles) {
          if (df_status s = best_of([&] { return run_half(tn); }, &ms)) return s;
          if (ms < best) {
            best = ms;
            tu.half_n = tn;
          }
        }
        if (df_status s = run_half(tu.half_n)) return s;
        best = 3.0e38f;
        for (int kt : kKTiles)
          for (int kr : kKRounds) {
            if (df_status s = best_of([&] { return run_k(kt, kr); }, &ms)) return s;
            if (ms < best) {
              best = ms;
              tu.k_tile = kt;
              tu.k_rounds = kr;
            }
          }
        return DF_OK;
      };
      const df_status ts = tune_all();
      c->timing = timing;
      c->ev_pool.push_back(ea);
      c->ev_pool.push_back(eb);
      if (ts != DF_OK) return ts;
      c->tune[c->arch + "|" + key] = tu;
      if (!c->cache_path.empty()) {
        // merge with what other processes wrote meanwhile, then rewrite; a cache that cannot be
        // written costs only the next process a tuning call
        std::string err;
        const BatchedTune mine = tu;
        if (std::ifstream(c->cache_path).good()) (void)tune_read(c, c->cache_path, &err);
        c->tune[c->arch + "|" + key] = mine;
        (void)tune_write(c, c->cache_path, &err);
      }
    }
  }
  if (df_status s = run_half(tu.half_n)) return s;
  if (df_status s = run_k(tu.k_tile, tu.k_rounds)) return s;
  // per problem: J-vectors and J, active-space blocks
  for (int i : order) {
    const df_problem& q = probs[i];
    const BatchedPiece& b = pc[(size_t)i];
    const int64_t ncol = batched_ncol(q);
    if (ncol == 0 || !(q.J || q.K || q.eri || q.papa)) continue;
    const double* Xo = (const double*)(ws + b.xo);
    const double* Xa = (const double*)(ws + b.xa);
    if (q.J && q.nocc > 0)
      if (df_status s = batched_coulomb(c, q, Xo, (double*)(ws + b.v), (double*)(ws + b.jp), (double*)(ws + b.dfull),
                                        (double*)(ws + b.dw), b.vsplit, (double*)(ws + b.vpart)))
        return s;
    if (q.eri && q.nac > 0) {
      double* buv = (double*)(ws + b.buv);
      if (df_status s = run_mo(c, q.Cact, q.nac, Xa, q.naux, q.nao, q.nac, buv)) return s;
      if (df_status s = run_pgemm(c, DF_KERNEL_ERI, buv, q.nac * q.nac, buv, q.nac * q.nac, q.naux, q.eri)) return s;
    }
    if (q.papa && q.nac > 0 && q.np > 0) {
      double* bpu = (double*)(ws + b.bpu);
      if (df_status s = run_mo(c, q.Cp, q.np, Xa, q.naux, q.nao, q.nac, bpu)) return s;
      if (df_status s = run_pgemm(c, DF_KERNEL_PAPA, bpu, q.np * q.nac, bpu, q.np * q.nac, q.naux, q.papa)) return s;
    }
  }
  // (pq|uv) through the AO basis, problem after problem in one region
  for (int i : order) {
    const df_problem& q = probs[i];
    if (!wants_ppaa(q)) continue;
    Plan pp;
    const PpaaPlan p = plan_ppaa(pp, q.naux, q.nao, q.nac, q.np);
    if (df_status s = ppaa_run(c, ws + ppaa_off, p, q.B, q.naux, q.nao, q.Cp, q.np, q.Cp, q.np, q.Cact, q.nac,
                               q.ppaa))
      return s;
  }
  return DF_OK;
}

// One problem of df_batched_step_split, its workspace at ws.
static df_status split_problem_run(df_ctx* c, char* ws, const df_problem& q, const int8_t* Bs, const int* Be,
                                   int nslice, bool k_fp64) {
  Plan pl;
  const SplitPiece b = plan_split_piece(pl, q, nslice, k_fp64);
  const int64_t ncol = batched_ncol(q), no = q.ndm * q.nocc, nao = q.nao, naux = q.naux, nac = q.nac;
  if (q.nocc == 0) {
    if (q.J) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(q.J, q.ndm * nao * nao, c->stream), "fill");
    if (q.K) DF_LAUNCH(DF_KERNEL_OTHER, dfk::launch_fill_zero(q.K, q.ndm * nao * nao, c->stream), "fill");
  }
  if (ncol == 0 || !(q.J || q.K || q.eri || q.papa)) return DF_OK;
  auto planes = [&](const SplitBuf& sb) { return (int8_t*)(ws + sb.planes); };
  auto exps = [&](const SplitBuf& sb) { return (int*)(ws + sb.ex); };
  const int64_t kpo = dfk::kpad64(nao);
  // half transform against the split b^P: [Cact | C_1 .. C_ndm] -> X_act AO-major, X_occ P-major
  double* cc = (double*)(ws + b.cc);
  std::vector<ColBlock> blks = {{q.Cact, nac, nac, 0}};
  for (int64_t z = 0; z < q.ndm; ++z) blks.push_back({q.Cocc + z * nao * q.nocc, q.nocc, q.nocc, nac + z * q.nocc});
  if (df_status s = pad_operand_plain(c, cc, nao, ncol, blks.data(), (int)blks.size())) return s;
  DF_LAUNCH(DF_KERNEL_SPLIT,
            dfk::launch_split_rows(dfk::op_map(cc, ncol, 1, nao, ncol), nao, nslice, planes(b.cs), exps(b.cs), c->stream),
            "split launch");
  double* Xo = (double*)(ws + b.xo);
  double* Xa = (double*)(ws + b.xa);
  dfk::OutMap OX = dfk::out_plain(Xa, naux * nao, ncol, naux * nac);
  OX.ml = nao;
  OX.s_mh = nac;
  OX.nsplit = nac;
  OX.p2 = Xo;
  OX.s2_m = no;
  DF_LAUNCH(DF_KERNEL_HALF_TRANSFORM,
            dfk::launch_slice_gemm(Bs, Be, naux * nao, planes(b.cs), exps(b.cs), ncol, kpo, nslice, OX, false, 1,
                                   nullptr, c->stream),
            "slice product launch");
  if (q.J && q.nocc > 0)
    if (df_status s = batched_coulomb(c, q, Xo, (double*)(ws + b.v), (double*)(ws + b.jp), (double*)(ws + b.dfull),
                                      (double*)(ws + b.dw), b.vsplit, (double*)(ws + b.vpart)))
      return s;
  if (q.K && q.nocc > 0 && k_fp64) {
    // K_z = sum_{P, i} X[P][m][z i] X[P][n][z i] in FP64, lower tiles, reduced and mirrored
    dfk::OpMap A = dfk::op_map(Xo, nao, no, q.nocc, 1);
    A.kb_n = naux;
    A.s_kb = nao * no;
    A.s_z = q.nocc;
    double* kpart = (double*)(ws + b.kpart);
    DF_LAUNCH(DF_KERNEL_K_SYRK, dfk::launch_syrk_partial(A, A, nao, q.ndm, b.nsk, kpart, c->stream), "K tiles launch");
    DF_LAUNCH(DF_KERNEL_K_REDUCE, dfk::launch_syrk_reduce(kpart, b.nsk, nao, q.ndm, q.K, c->stream),
              "K reduce launch");
  } else if (q.K && q.nocc > 0) {
    // rows m of each density's X_occ over (P, i), then K_z = sum_{P, i} X[P][m][z i] X[P][n][z i]
    // for all densities in one batched launch, lower tiles, reduced and mirrored
    int8_t* xs = planes(b.xos);
    int* xe = exps(b.xos);
    // every density's rows in one launch set: density z at Xo + z nocc
    dfk::OpMap ox = dfk::op_map(Xo, nao, no, q.nocc, 1);
    ox.kb_n = naux;
    ox.s_kb = nao * no;
    ox.s_z = q.nocc;
    DF_LAUNCH(DF_KERNEL_SPLIT,
              dfk::launch_split_rows_batched(ox, naux * q.nocc, nslice, xs, xe, q.ndm, b.xplane, nao, c->stream),
              "split launch");
    double* kpart = (double*)(ws + b.kpart);
    const dfk::SliceBatch zs{b.xplane, nao, b.xplane, nao};
    DF_LAUNCH(DF_KERNEL_K_SYRK,
              dfk::launch_slice_gemm_batched(xs, xe, nao, xs, xe, nao, dfk::kpad64(naux * q.nocc), nslice,
                                             dfk::out_plain(kpart, nao, nao, nao), true, b.nsk, kpart, q.ndm, zs,
                                             c->stream),
              "slice product launch");
    DF_LAUNCH(DF_KERNEL_K_REDUCE, dfk::launch_syrk_reduce(kpart, b.nsk, nao, q.ndm, q.K, c->stream),
              "K reduce launch");
  }
  const bool de = q.eri && nac > 0, dp = q.papa && nac > 0 && q.np > 0;
  if (de || dp) {
    // rows (P, u) of X_act over m; b^P_{lu} = sum_m Cl[m][l] X[m][P][u] for l in Cact, Cp
    const dfk::OpMap oxa = dfk::op_map(Xa, naux * nac, 1, nao, naux * nac);
    DF_LAUNCH(DF_KERNEL_SPLIT, dfk::launch_split_rows(oxa, nao, nslice, planes(b.xas), exps(b.xas), c->stream),
              "split launch");
    auto second = [&](const double* Cl, int64_t nl, const SplitBuf& sb, double* out) -> df_status {
      DF_LAUNCH(DF_KERNEL_SPLIT,
                dfk::launch_split_rows(dfk::op_map(Cl, nl, 1, nao, nl), nao, nslice, planes(sb), exps(sb), c->stream),
                "split launch");
      dfk::OutMap O = dfk::out_plain(out, nl, naux * nac, nac);
      O.nl = nac;
      O.s_nh = nl * nac;
      DF_LAUNCH(DF_KERNEL_MO_TRANSFORM,
                dfk::launch_slice_gemm(planes(sb), exps(sb), nl, planes(b.xas), exps(b.xas), naux * nac, kpo, nslice,
                                       O, false, 1, nullptr, c->stream),
                "slice product launch");
      return DF_OK;
    };
    // sum over P of products of rows (l, u) of b^P_lu, split along P
    auto pproduct = [&](int kind, double* bl, int64_t rows, const SplitBuf& sb, double* out) -> df_status {
      DF_LAUNCH(DF_KERNEL_SPLIT,
                dfk::launch_split_rows(dfk::op_map(bl, rows, 1, naux, rows), naux, nslice, planes(sb), exps(sb),
                                       c->stream),
                "split launch");
      DF_LAUNCH(kind,
                dfk::launch_slice_gemm(planes(sb), exps(sb), rows, planes(sb), exps(sb), rows, dfk::kpad64(naux), nslice,
                                       dfk::out_plain(out, rows, rows, rows), false, 1, nullptr, c->stream),
                "slice product launch");
      return DF_OK;
    };
    if (de) {
      double* buv = (double*)(ws + b.buv);
      if (df_status s = second(q.Cact, nac, b.cas, buv)) return s;
      if (df_status s = pproduct(DF_KERNEL_ERI, buv, nac * nac, b.buvs, q.eri)) return s;
    }
    if (dp) {
      double* bpu = (double*)(ws + b.bpu);
      if (df_status s = second(q.Cp, q.np, b.cps, bpu)) return s;
      if (df_status s = pproduct(DF_KERNEL_PAPA, bpu, q.np * nac, b.bpus, q.papa)) return s;
    }
  }
  return DF_OK;
}

df_status df_batched_split_workspace_size(const df_problem* probs, int nprob, int nslice, int flags, size_t* bytes) {
  if (!bytes || nprob < 0 || (nprob > 0 && !probs)) return DF_ERR_ARG;
  *bytes = 0;
  if (flags & ~DF_SPLIT_K_FP64) return DF_ERR_UNSUPPORTED;
  if (nslice < 4 || nslice > 8) return DF_ERR_SHAPE;
  for (int i = 0; i < nprob; ++i) {
    const df_problem& q = probs[i];
    if (q.naux < 1 || q.nao < 1 || q.nao > kMaxNao || q.ndm < 1 || q.ndm > 65535 || q.nocc < 0 || q.nac < 0 ||
        q.np < 0)
      return DF_ERR_SHAPE;
    Plan pl;
    plan_split_piece(pl, q, nslice, (flags & DF_SPLIT_K_FP64) != 0);
    *bytes = std::max(*bytes, pl.total);
  }
  *bytes = std::max(*bytes, batched_ppaa_bytes(probs, nprob));
  return DF_OK;
}

df_status df_batched_step_split(df_ctx* ctx, const df_problem* probs, const int8_t* const* Bs, const int* const* Be,
                                int nprob, int nslice, int flags) {
  df_ctx* c = ctx;
  if (check_ctx(c)) return DF_ERR_ARG;
  if (flags & ~DF_SPLIT_K_FP64) return fail(c, DF_ERR_UNSUPPORTED, "df_batched_step_split: unknown flags");
  const bool k_fp64 = (flags & DF_SPLIT_K_FP64) != 0;
  if (nslice < 4 || nslice > 8) return fail(c, DF_ERR_SHAPE, "nslice must be in [4, 8]");
  if (nprob < 0 || (nprob > 0 && (!probs || !Bs || !Be))) return fail(c, DF_ERR_ARG, "probs, Bs or Be is NULL");
  std::vector<Range> rs;
  size_t need = 0;
  for (int i = 0; i < nprob; ++i) {
    const df_problem& q = probs[i];
    const std::string tag = "problem " + std::to_string(i) + " ";
    if (df_status s = check_core(c, q.B, q.naux, q.nao)) return s;
    if (q.ndm < 1 || q.ndm > 65535 || q.nocc < 0 || q.nac < 0 || q.np < 0)
      return fail(c, DF_ERR_SHAPE, tag + "has a bad size");
    if (dfk::rpad32(q.naux * q.nao) > 0x7fffffffLL || dfk::rpad32(q.naux * q.nac) > 0x7fffffffLL ||
        dfk::rpad32(q.np * q.nac) > 0x7fffffffLL || q.naux * q.nocc > (1LL << 30))
      return fail(c, DF_ERR_SHAPE, tag + "is too large for the split path");
    if (q.nocc > 0 && (q.J || q.K) && !q.Cocc) return fail(c, DF_ERR_ARG, tag + "Cocc is NULL");
    if (q.nac > 0 && (q.eri || q.papa) && !q.Cact) return fail(c, DF_ERR_ARG, tag + "Cact is NULL");
    if (q.np > 0 && q.papa && !q.Cp) return fail(c, DF_ERR_ARG, tag + "Cp is NULL");
    if (wants_ppaa(q) && (!q.Cact || !q.Cp)) return fail(c, DF_ERR_ARG, tag + "ppaa needs Cact and Cp");
    if (!Bs[i] || !Be[i]) return fail(c, DF_ERR_ARG, tag + "Bs or Be is NULL");
    if ((uintptr_t)Bs[i] % 16 != 0) return fail(c, DF_ERR_ARG, tag + "Bs must be 16-byte aligned");
    const int64_t npair = q.nao * (q.nao + 1) / 2;
    rs.push_back({q.B, dbytes(q.naux * npair), "B", false});
    rs.push_back({Bs[i], (size_t)dfk::split_plane_bytes(q.naux * q.nao, q.nao, nslice), "Bs", false});
    rs.push_back({Be[i], (size_t)q.naux * q.nao * 4, "Be", false});
    rs.push_back({q.Cocc, dbytes(q.ndm * q.nao * q.nocc), "Cocc", false});
    rs.push_back({q.Cact, dbytes(q.nao * q.nac), "Cact", false});
    rs.push_back({q.Cp, dbytes(q.nao * q.np), "Cp", false});
    rs.push_back({q.J, dbytes(q.ndm * q.nao * q.nao), "J", true});
    rs.push_back({q.K, dbytes(q.ndm * q.nao * q.nao), "K", true});
    rs.push_back({q.eri, dbytes(q.nac * q.nac * q.nac * q.nac), "eri", true});
    rs.push_back({q.papa, dbytes(q.np * q.nac * q.np * q.nac), "papa", true});
    rs.push_back({q.ppaa, dbytes(q.nac * (q.nac + 1) / 2 * q.np * q.np), "ppaa", true});
    Plan pl;
    plan_split_piece(pl, q, nslice, k_fp64);
    need = std::max(need, pl.total);
  }
  need = std::max(need, batched_ppaa_bytes(probs, nprob));
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (df_status s = need_ws(c, need)) return s;
  if (need) rs.push_back({c->ws, need, "workspace", true});
  if (!check_overlap(c, rs)) return DF_ERR_ARG;
  if (nprob == 0) return DF_OK;
  if (df_status s = enter(c)) return s;
  for (int i = 0; i < nprob; ++i) {
    const df_problem& q = probs[i];
    if (df_status s = split_problem_run(c, c->ws, q, Bs[i], Be[i], nslice, k_fp64)) return s;
    if (wants_ppaa(q)) {
      // (pq|uv) in FP64 through the AO basis, in the same region
      Plan pp;
      const PpaaPlan p = plan_ppaa(pp, q.naux, q.nao, q.nac, q.np);
      if (df_status s = ppaa_run(c, c->ws, p, q.B, q.naux, q.nao, q.Cp, q.np, q.Cp, q.np, q.Cact, q.nac, q.ppaa))
        return s;
    }
  }
  return DF_OK;
}

}  // extern "C"
