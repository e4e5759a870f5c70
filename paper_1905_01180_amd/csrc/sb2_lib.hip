// libsb2: C ABI of the second-Born self-energy / GKBA collision-integral path.
//
// Contraction chain (Eq. 13 regrouped; Eq. 19 / Fig. 2 give the paper's own
// path, this is another valid one).  With w_mqsj = 2 v_mqsj - v_qmsj,
//   Sigma_ij = sum v_irpn w_mqsj G_nm G_pq Gbar_sr
// is evaluated per slice (pair of times, kind <>) as four contractions in which
// both operands are contiguous along the summed index:
//   R1  A[n][j][s][q] = sum_m G_nm  W_T[j][s][q][m]              (slices stacked: rows 2S N)
//   R2  B[n][p][j][s] = sum_q G_pq  A[n][j][s][q]                (batched over (slice, n))
//   R3  C[j][n][p][r] = sum_s B[n][p][j][s] GbT[r][s]            (batched over slices)
//   R4  Sigma_ij      = sum_{(n,p,r)} Vp[i][n][p][r] C[j][n][p][r]   (split-K, float64 partials)
// with the interaction laid out once per call as W_T[j][s][q][m] = w_mqsj and
// Vp[i][n][p][r] = v_irpn, and GbT[r][s] = Gbar_sr.  R1 and R4 share W_T / Vp
// across all slices of a chunk of past times; the intermediates A/C and B each
// take 2S N^4 complex entries.  Each stage is one k_stream launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <initializer_list>
#include <map>
#include <mutex>
#include <vector>

#include "kernels.hpp"
#include "chain.hpp"
#include "group.hpp"
#include "sb2.h"

using namespace sb2;

namespace {

constexpr size_t ALIGN = 256;
inline size_t al(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }
constexpr size_t C128 = 16;                       // bytes of one complex float64
constexpr size_t INTERMEDIATE_BUDGET = 32ull << 30;  // bytes for the two chain intermediates


inline bool prec_ok(int p) { return p == SB2_FP64 || p == SB2_FP32 || p == SB2_SPLIT_FP16; }
// SB2_SPLIT_BF16 is a known precision that no entry point implements
inline int prec_status(int p) { return prec_ok(p) ? SB2_OK : (p == SB2_SPLIT_BF16 ? SB2_EUNSUPPORTED : SB2_EINVAL); }
inline size_t bulk_bytes(int p) { return p == SB2_FP64 ? 8 : 4; }   // one real scalar of the bulk type

GemmArgs gdef() {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.nbl = 1;
  g.alpha_re = 1.0;
  g.kpromote = 4;
  return g;
}

// ---------------------------------------------------------------------------
// GEMM launchers
// ---------------------------------------------------------------------------
template <typename T, typename OutT, int WM, int WN, int FM, int FN, bool AC, bool BC, bool ACC64>
hipError_t launch_f(GemmArgs g, int nbatch, hipStream_t s) {
  constexpr int BM = 16 * FM * WM, BN = 16 * FN * WN;
  if (g.kchunk <= 0) g.kchunk = g.K > 0 ? g.K : 1;
  g.tiles_m = (g.M + BM - 1) / BM;
  const int tiles_n = (g.N + BN - 1) / BN;
  const int nz = g.K > 0 ? (g.K + g.kchunk - 1) / g.kchunk : 1;
  dim3 grid(g.tiles_m * tiles_n, nbatch, nz);
  hipLaunchKernelGGL((k_gemm<T, OutT, WM, WN, FM, FN, AC, BC, ACC64>), grid, dim3(64 * WM * WN), 0, s, g);
  return hipGetLastError();
}

template <typename OutT, int WM, int WN, int FM, int FN, bool AC, bool BC, bool ACC64>
hipError_t launch_h(GemmArgs g, int nbatch, hipStream_t s) {
  constexpr int BM = 16 * FM * WM, BN = 16 * FN * WN;
  if (g.kchunk <= 0) g.kchunk = g.K > 0 ? g.K : 1;
  g.tiles_m = (g.M + BM - 1) / BM;
  const int tiles_n = (g.N + BN - 1) / BN;
  const int nz = g.K > 0 ? (g.K + g.kchunk - 1) / g.kchunk : 1;
  dim3 grid(g.tiles_m * tiles_n, nbatch, nz);
  hipLaunchKernelGGL((k_gemm_h16<OutT, WM, WN, FM, FN, AC, BC, ACC64>), grid, dim3(64 * WM * WN), 0, s, g);
  return hipGetLastError();
}

// float64 complex x complex, small-M shape (N x N products, propagators, collision terms)
hipError_t zgemm(GemmArgs g, int nbatch, hipStream_t s) {
  return launch_f<double, double, 1, 4, 7, 1, true, true, false>(g, nbatch, s);
}

// ---------------------------------------------------------------------------
// Workspace plans
// default workgroups per single-slab stage launch: float64 / float32, and
// split float16 (more, smaller column ranges per workgroup: its first
// contraction is 5-10 % faster with 3072 than with 768 at N = 48 .. 128)
constexpr int PERSIST_TARGET = 768;
constexpr int PERSIST_TARGET_H16 = 3072;

constexpr int R23_WGS = 512;          // default workgroups of the fused second/third contraction
constexpr int R23_MAX_N = 112;        // largest N of the fused kernel (LDS holds Gbar and one A slab)

// Autotuned launch parameters per (N, precision): workgroups per single-slab
// stage launch, the R4 split-K factor (percent of the default count) and the
// workgroups of the fused R2+R3 kernel (split float16, N <= 112; 0 = run R2
// and R3 as separate stages).
struct TuneCfg { int persist = PERSIST_TARGET; int r4pct = 100; int r23 = R23_WGS; };
std::map<std::pair<int, int>, TuneCfg> g_tune;
TuneCfg default_tune(int prec) {
  TuneCfg tc;
  if (prec == SB2_SPLIT_FP16) tc.persist = PERSIST_TARGET_H16;
  return tc;
}
TuneCfg tune_of(int N, int prec) {
  auto it = g_tune.find({N, prec});
  return it == g_tune.end() ? default_tune(prec) : it->second;
}

// ---------------------------------------------------------------------------
struct ChainPlan {
  int N = 0, S = 0, nz = 1, kchunk = 1;
  i64 KpW = 0, KpV = 0;                 // row pitches of W_T and Vp
  // n-chunked layout (split float16 with the fused second/third contraction):
  // Vp[i][n KB + (p N + r)] with KB = N^2 rounded up to 8 (zero padding), C
  // stored as [n][(b, j)][(p, r)], and the last contraction split into the N
  // chunks n
  bool chunked = false;
  i64 KB = 0;
  size_t w = 0, vp = 0, gs = 0, gbs = 0, x1 = 0, x2 = 0, part = 0, scal = 0, end = 0;
};

inline int slab_depth(int prec) { return prec == SB2_SPLIT_FP16 ? 128 : prec == SB2_FP32 ? 64 : 32; }
inline size_t inter_bytes(int prec) { return prec == SB2_SPLIT_FP16 ? 4 : bulk_bytes(prec); }  // W_T / Vp per element

// R4 split-K: about 2048 * scale workgroups (enough to fill the chip at scale
// 1), chunk a multiple of the slab depth.
void r4_split(int N, int ns, int prec, int& nz, int& kchunk, double scale = 1.0) {
  const long long K = (long long)N * N * N;
  const int bk = slab_depth(prec);
  const long long coltiles = ((long long)ns * N + 63) / 64;
  const long long rowtiles = (N + 111) / 112;
  const long long target = (long long)(2048.0 * scale + 0.5);
  long long want = (target + coltiles * rowtiles - 1) / (coltiles * rowtiles);
  const long long maxz = (K + bk - 1) / bk;
  if (want < 1) want = 1;
  if (want > maxz) want = maxz;
  if (want > 4096) want = 4096;
  long long kc = (K + want - 1) / want;
  kc = (kc + bk - 1) / bk * bk;
  kchunk = (int)kc;
  nz = (int)((K + kc - 1) / kc);
}

// share: this chain's part of a grouped launch (1 when it runs alone); scales
// the R4 split so that the whole launch, not each member, fills the chip.
ChainPlan chain_plan(int N, int pairs, int prec, size_t base, int forceS = 0, double share = 1.0,
                     bool allow_chunked = true) {
  ChainPlan p;
  p.N = N;
  const size_t n4 = (size_t)N * N * N * N, n3 = (size_t)N * N * N, n2 = (size_t)N * N;
  const size_t bb = bulk_bytes(prec);
  const size_t per_pair = 2 * 2 * n4 * 2 * bb;      // two buffers x two slices x N^4 complex
  size_t S = forceS > 0 ? (size_t)forceS : INTERMEDIATE_BUDGET / per_pair;
  if (S < 1) S = 1;
  if (S > (size_t)pairs) S = pairs;
  const size_t smax = 65535 / (2 * (size_t)N);       // R2 batch = 2 S N workgroup rows in grid.y
  if (S > smax) S = smax;
  p.S = (int)S;
  p.KpW = (N + 7) / 8 * 8;
  p.KpV = ((i64)n3 + 7) / 8 * 8;
  p.KB = ((i64)n2 + 7) / 8 * 8;
  int nz_max, kc_max;
  r4_split(N, 2 * p.S, prec, nz_max, kc_max, 2.0);
  r4_split(N, 2 * p.S, prec, p.nz, p.kchunk, tune_of(N, prec).r4pct / 100.0 * share);
  if (p.nz > nz_max) nz_max = p.nz;
  // buffer sizes cover both layouts, so they do not depend on tuned values
  const bool h16 = prec == SB2_SPLIT_FP16;
  if (h16 && nz_max < N) nz_max = N;
  const i64 vrow = h16 ? std::max(p.KpV, (i64)N * p.KB) : p.KpV;
  p.chunked = allow_chunked && h16 && N <= R23_MAX_N && tune_of(N, prec).r23 > 0;
  if (p.chunked) {
    p.KpV = (i64)N * p.KB;
    p.nz = N;
    p.kchunk = (int)n2;
  }
  const size_t ib = inter_bytes(prec);
  size_t o = base;
  p.scal = o; o += al((S_TRASH + S_TRASH_WORDS) * 4);
  p.w = o; o += al(n3 * (size_t)p.KpW * ib);
  p.vp = o; o += al((size_t)N * (size_t)vrow * ib);
  p.gs = o; o += al(2 * S * n2 * 2 * bb);
  p.gbs = o; o += al(2 * S * n2 * 2 * bb);
  // (+64 bytes: the last contraction may read up to 7 elements past a row end)
  p.x1 = o; o += al(2 * S * n4 * 2 * bb + 64);
  p.x2 = o; o += al(2 * S * n4 * 2 * bb + 64);
  p.part = o; o += al((size_t)nz_max * N * 2 * S * N * C128);
  p.end = o;
  return p;
}

struct CollPlan {
  size_t U, X, Y, Gl, Gg, Glb, Ggb, Sl, Sg, terms, ex1, ex2;
  ChainPlan ch;
  size_t end;
};

CollPlan coll_plan(int N, int T, int prec, int forceS = 0, double share = 1.0, bool allow_chunked = true) {
  CollPlan c;
  const size_t hist = (size_t)T * N * N * C128;
  size_t o = 0;
  c.U = o; o += al(hist);
  c.X = o; o += al(hist);
  c.Y = o; o += al(hist);
  c.Gl = o; o += al(hist);
  c.Gg = o; o += al(hist);
  c.Glb = o; o += al(hist);
  c.Ggb = o; o += al(hist);
  c.Sl = o; o += al(hist);
  c.Sg = o; o += al(hist);
  c.terms = o; o += al(hist);
  c.ex1 = o; o += al((size_t)N * N * C128);
  c.ex2 = o; o += al((size_t)N * N * C128);
  c.ch = chain_plan(N, T, prec, o, forceS, share, allow_chunked);
  c.end = c.ch.end;
  return c;
}

// Autotuning workload: the first chunk of past times (at most S), and its
// workspace: that evaluation's plus one N x N output at the end.
int tune_len(int N, int T, int prec) {
  const int S = coll_plan(N, T, prec).ch.S;
  return S < T ? S : T;
}
size_t tune_bytes(int N, int T, int prec) {
  return al(coll_plan(N, tune_len(N, T, prec), prec).end) + al((size_t)N * N * C128);
}

size_t rho_plan(int N) { return 4 * al((size_t)N * N * C128); }

// Workspace of the special-vertex collision integrals: the GKBA history and
// self-energy areas of coll_plan (no contraction chain), and for the symmetric
// basis the float64 operands of the bubble and exchange products for a chunk
// of past times (the exchange operand holds N^3 per slice).
struct VertPlan {
  size_t U, X, Y, Gl, Gg, Glb, Ggb, Sl, Sg, terms, ex1, ex2, Vc, P, Q, R, A, B, end;
  int chunk;
};
VertPlan vert_plan(int N, int T, int vertex) {
  VertPlan p;
  const size_t m = al((size_t)N * N * C128), hist = al((size_t)T * N * N * C128);
  size_t o = 0;
  p.U = o; o += hist;
  p.X = o; o += hist;
  p.Y = o; o += hist;
  p.Gl = o; o += hist;
  p.Gg = o; o += hist;
  p.Glb = o; o += hist;
  p.Ggb = o; o += hist;
  p.Sl = o; o += hist;
  p.Sg = o; o += hist;
  p.terms = o; o += hist;
  p.ex1 = o; o += m;
  p.ex2 = o; o += m;
  p.chunk = 0;
  p.Vc = p.P = p.Q = p.R = p.A = p.B = o;
  if (vertex == SB2_VERTEX_SYMMETRIC) {
    const size_t n3 = (size_t)N * N * N * C128;
    long long ch = (long long)((size_t(1) << 29) / n3);
    p.chunk = (int)(ch < 1 ? 1 : (ch > T ? T : ch));
    p.Vc = o; o += m;
    p.P = o; o += al((size_t)p.chunk * N * N * C128);
    p.Q = o; o += al((size_t)p.chunk * N * N * C128);
    p.R = o; o += al((size_t)p.chunk * N * N * C128);
    p.A = o; o += al((size_t)p.chunk * n3);
    p.B = o; o += al((size_t)p.chunk * n3);
  }
  p.end = o;
  return p;
}



// Workspace of a propagation that ends with n_end + 1 densities: the
// collision evaluations (at most n_end - 1 past times; the collision plan
// grows with T; vertex != 0: the special-vertex plan) followed by the step's
// own N x N matrices and the staging area of the propagator-history update.
struct PropPlan {
  size_t heff, ustep, hqp, uqp, I, T1, ex1, ex2, tmp, end;
};
PropPlan prop_plan(int N, int n_end, int prec, int vertex = 0) {
  PropPlan p;
  const size_t m = al((size_t)N * N * C128);
  size_t o = 0;
  if (n_end >= 2) o = al(vertex ? vert_plan(N, n_end - 1, vertex).end : coll_plan(N, n_end - 1, prec).end);
  p.heff = o; o += m;
  p.ustep = o; o += m;
  p.hqp = o; o += m;
  p.uqp = o; o += m;
  p.I = o; o += m;
  p.T1 = o; o += m;
  p.ex1 = o; o += m;
  p.ex2 = o; o += m;
  p.tmp = o; o += al((size_t)(n_end > 1 ? n_end - 1 : 1) * N * N * C128);
  p.end = o;
  return p;
}

inline char* at(void* ws, size_t off) { return reinterpret_cast<char*>(ws) + off; }

// ---------------------------------------------------------------------------
// Optional stage timing with HIP events recorded on the launch stream (off by
// default; used by the benchmark).  Slots: 0..3 = R1..R4, 4 = interaction
// layout, 5 = propagators + GKBA, 6 = operand packing + split-K reduction,
// 7 = collision terms + sum over past times.
// ---------------------------------------------------------------------------
constexpr int NSLOTS = 8;
struct ProfRec { int slot; hipEvent_t a, b; };
struct Prof {
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};
Prof g_prof;

struct StageTimer {
  hipEvent_t b_ = nullptr;
  hipStream_t s_;
  int slot_;
  hipEvent_t a_ = nullptr;
  StageTimer(int slot, hipStream_t s) : s_(s), slot_(slot) {
    if (!g_prof.on) return;
    a_ = g_prof.get();
    b_ = g_prof.get();
    if (a_ && b_) (void)hipEventRecord(a_, s_);
  }
  ~StageTimer() {
    if (!g_prof.on || !a_ || !b_) return;
    (void)hipEventRecord(b_, s_);
    g_prof.recs.push_back({slot_, a_, b_});
  }
};

#define SB2_TRY(expr)                      \
  do {                                     \
    hipError_t e_ = (expr);                \
    if (e_ != hipSuccess) return SB2_EHIP; \
  } while (0)

inline int blocks(long long n, int bs) { return (int)((n + bs - 1) / bs); }

#define SB2_PREC(p)                          \
  do {                                       \
    const int ps_ = prec_status(p);          \
    if (ps_ != SB2_OK) return ps_;           \
  } while (0)

// An error left by an earlier asynchronous failure is reported (and cleared)
// by the next entry point that enqueues work.
#define SB2_ENTRY()                                         \
  do {                                                      \
    if (hipGetLastError() != hipSuccess) return SB2_EHIP;   \
  } while (0)

// ---------------------------------------------------------------------------
// Optional input checks, run when the environment has SB2_CHECK=1: every
// input finite, h and the density matrices Hermitian to 1e-10 relative.  They
// synchronise the stream (a device-to-host copy of three words at `scr`, the
// start of the call's scratch memory, before any work is enqueued), so they
// are off the hot path and not for use under stream capture.
// ---------------------------------------------------------------------------
bool check_on() {
  const char* e = std::getenv("SB2_CHECK");
  return e && e[0] == '1' && e[1] == 0;
}

struct CheckItem {
  int kind;          // 0: N x N complex matrices that must be Hermitian, 1: finite complex, 2: finite real
  const void* p;
  i64 count;         // matrices (kind 0) or scalars (kinds 1, 2)
};

int run_checks(hipStream_t s, void* scr, int N, std::initializer_list<CheckItem> items) {
  unsigned* out = reinterpret_cast<unsigned*>(scr);
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, out, 3, 0u);
  for (const CheckItem& it : items) {
    if (!it.p || it.count < 1) continue;
    if (it.kind == 0) {
      const i64 n = it.count * N * N;
      hipLaunchKernelGGL(k_check_herm, dim3(blocks(n, 256)), dim3(256), 0, s, N, it.count,
                         reinterpret_cast<const cplx*>(it.p), out);
    } else {
      const i64 n = it.kind == 1 ? 2 * it.count : it.count;
      hipLaunchKernelGGL(k_check_finite, dim3(blocks(n, 256)), dim3(256), 0, s, n,
                         reinterpret_cast<const double*>(it.p), out);
    }
    if (hipGetLastError() != hipSuccess) return SB2_EHIP;
  }
  unsigned host[3] = {0, 0, 0};
  if (hipMemcpyAsync(host, out, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess) return SB2_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return SB2_EHIP;
  float herm, mx;
  std::memcpy(&herm, &host[0], 4);
  std::memcpy(&mx, &host[1], 4);
  if (host[2] != 0) return SB2_ECHECK;
  if ((double)herm > 1e-10 * std::max(1.0, (double)mx)) return SB2_ECHECK;
  return SB2_OK;
}

#define SB2_CHECKS(scr, N, ...)                                               \
  do {                                                                        \
    if (check_on()) {                                                         \
      const int cs_ = run_checks(reinterpret_cast<hipStream_t>(stream), (scr), (N), {__VA_ARGS__}); \
      if (cs_ != SB2_OK) return cs_;                                          \
    }                                                                         \
  } while (0)

// ---------------------------------------------------------------------------
// The chain for one chunk of ns slices
// ---------------------------------------------------------------------------
// v: the dense tensor, or (PACKED) its 8-fold packed values (Eq. 4)
template <typename T, bool PACKED>
hipError_t prep_interaction(int N, const double* v, const ChainPlan& p, void* ws, int prec, hipStream_t s) {
  unsigned* scal = reinterpret_cast<unsigned*>(at(ws, p.scal));
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, scal, (int)S_NWORDS, 0u);
  const bool h = prec == SB2_SPLIT_FP16;
  if (h) hipLaunchKernelGGL(k_max_vw<PACKED>, dim3(N * N), dim3(256), 0, s, N, v, scal + S_VMAX, scal + S_WMAX);
  const int nj = (N + 15) / 16, nm = (N + 7) / 8;
  const i64 planeW = (i64)N * N * N * p.KpW, planeV = (i64)N * p.KpV;
  hipLaunchKernelGGL((k_prep_wt<T, PACKED>), dim3(N * nj * nm), dim3(256), 0, s, N, (int)p.KpW, v,
                     reinterpret_cast<T*>(at(ws, p.w)), planeW, h ? scal + S_WMAX : nullptr);
  if (p.chunked) {                               // zero n-block padding
    const long long words = (long long)N * p.KpV;  // two float16 planes: N KpV 32-bit words
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks(words, 256)), dim3(256), 0, s,
                       reinterpret_cast<unsigned*>(at(ws, p.vp)), (int)words, 0u);
  }
  hipLaunchKernelGGL((k_prep_vpt<T, PACKED>), dim3(N * N), dim3(256), 0, s, N, p.KpV, p.chunked ? p.KB : (i64)N * N, v,
                     reinterpret_cast<T*>(at(ws, p.vp)), planeV, h ? scal + S_VMAX : nullptr);
  return hipGetLastError();
}

ChainRefs chain_refs(int prec, int N, int ns, const ChainPlan& p, void* ws, void* cbuf) {
  ChainRefs r;
  r.N = N;
  r.ns = ns;
  r.prec = prec;
  r.kchunk = p.kchunk;
  r.KpW = p.KpW;
  r.KpV = p.KpV;
  r.Gs = at(ws, p.gs);
  r.GbT = at(ws, p.gbs);
  r.W = at(ws, p.w);
  r.Vp = at(ws, p.vp);
  r.X1 = at(ws, p.x1);
  r.X2 = at(ws, p.x2);
  r.C3 = cbuf;
  r.part = at(ws, p.part);
  r.scal = reinterpret_cast<unsigned*>(at(ws, p.scal));
  r.chunked = p.chunked ? 1 : 0;
  r.KB = p.KB;
  return r;
}

template <int PK, int STAGE, int FSN>
hipError_t launch_stage_fs(const ChainRefs& r, hipStream_t st) {
  int nbatch;
  StreamArgs g = stage_args(STAGE, r, nbatch);
  const StageGeom q = stage_geom<PK, STAGE, FSN>(g, nbatch, tune_of(r.N, r.prec).persist);
  const long long gx = (long long)q.tiles_s * q.npersist;
  dim3 grid((unsigned)gx, (unsigned)q.nbatch, (unsigned)q.nz);
  StageTimer tm(STAGE, st);
  hipLaunchKernelGGL((k_stage<PK, STAGE, FSN>), grid, dim3(64 * StageCfg<PK, STAGE>::NW), 0, st, g, q);
  return hipGetLastError();
}

// Stages 1-3: the shared tile's height follows N (stage_fs)
template <int PK, int STAGE>
hipError_t launch_stage(const ChainRefs& r, hipStream_t st) {
  if constexpr (STAGE == 0) {
    return launch_stage_fs<PK, 0, 0>(r, st);
  } else {
    switch (stage_fs(r.N)) {
      case 2: return launch_stage_fs<PK, STAGE, 2>(r, st);
      case 4: return launch_stage_fs<PK, STAGE, 4>(r, st);
      case 6: return launch_stage_fs<PK, STAGE, 6>(r, st);
      case 7: return launch_stage_fs<PK, STAGE, 7>(r, st);
      default: return launch_stage_fs<PK, STAGE, 8>(r, st);
    }
  }
}

template <int NT>
hipError_t launch_r23_nt(const ChainRefs& r, int nwg, hipStream_t st) {
  const R23Args a = r23_args(r);
  StageTimer tm(1, st);
  if (r.N % 2 == 0)
    hipLaunchKernelGGL((k_r23_h16<NT, true>), dim3(nwg), dim3(R23Cfg<NT>::NTH), 0, st, a);
  else
    hipLaunchKernelGGL((k_r23_h16<NT, false>), dim3(nwg), dim3(R23Cfg<NT>::NTH), 0, st, a);
  return hipGetLastError();
}

// Workgroups of a fused launch (tuned per N and precision).
inline long long r23_wgs(int N, int prec) { return tune_of(N, prec).r23; }

// Fused R2+R3 (split float16): A in X1 -> C in X2.
hipError_t launch_r23(const ChainRefs& r, long long nwg, hipStream_t st) {
  const long long ntask = (long long)r.ns * r.N * r.N;
  if (nwg > ntask) nwg = (int)ntask;
  switch ((r.N + 15) / 16) {
    case 1: return launch_r23_nt<1>(r, nwg, st);
    case 2: return launch_r23_nt<2>(r, nwg, st);
    case 3: return launch_r23_nt<3>(r, nwg, st);
    case 4: return launch_r23_nt<4>(r, nwg, st);
    case 5: return launch_r23_nt<5>(r, nwg, st);
    case 6: return launch_r23_nt<6>(r, nwg, st);
    case 7: return launch_r23_nt<7>(r, nwg, st);
    default: return hipErrorInvalidValue;
  }
}

template <int FS>
hipError_t launch_r4_fs(const ChainRefs& r, hipStream_t st) {
  const R4Args a = r4_args(r);
  StageTimer tm(3, st);
  const dim3 grid((unsigned)r4_tiles(a), (unsigned)r.N);
  if ((a.kc & 1) == 0) hipLaunchKernelGGL((k_r4_h16<FS, true>), grid, dim3(R4_THREADS), 0, st, a);
  else hipLaunchKernelGGL((k_r4_h16<FS, false>), grid, dim3(R4_THREADS), 0, st, a);
  return hipGetLastError();
}

// Last contraction, split float16, n-chunked layout (one chunk per n).
hipError_t launch_r4_h16(const ChainRefs& r, hipStream_t st) {
  switch ((r.N + 15) / 16) {
    case 1: return launch_r4_fs<1>(r, st);
    case 2: return launch_r4_fs<2>(r, st);
    case 3: return launch_r4_fs<3>(r, st);
    case 4: return launch_r4_fs<4>(r, st);
    case 5: return launch_r4_fs<5>(r, st);
    case 6: return launch_r4_fs<6>(r, st);
    case 7: return launch_r4_fs<7>(r, st);
    default: return hipErrorInvalidValue;
  }
}

// the plan decides: the n-chunked layout goes with the fused kernel
inline bool fused_r23(const ChainRefs& r) { return r.prec == SB2_SPLIT_FP16 && r.chunked && r.C3 == nullptr; }

template <int PK>
hipError_t run_chain_pk(const ChainRefs& r, hipStream_t st) {
  hipError_t e;
  if (PK == PK_H16 && fused_r23(r)) {
    if ((e = launch_stage<PK, 0>(r, st)) != hipSuccess) return e;
    if ((e = launch_r23(r, r23_wgs(r.N, r.prec), st)) != hipSuccess) return e;
    return launch_r4_h16(r, st);                      // the fused kernel leaves C in X2
  }
  if ((e = launch_stage<PK, 0>(r, st)) != hipSuccess) return e;
  if ((e = launch_stage<PK, 1>(r, st)) != hipSuccess) return e;
  if ((e = launch_stage<PK, 2>(r, st)) != hipSuccess) return e;
  return launch_stage<PK, 3>(r, st);
}

hipError_t run_chain(int prec, int N, int ns, const ChainPlan& p, void* ws, hipStream_t st, void* cbuf = nullptr) {
  const ChainRefs r = chain_refs(prec, N, ns, p, ws, cbuf);
  if (prec == SB2_FP64) return run_chain_pk<PK_F64>(r, st);
  if (prec == SB2_FP32) return run_chain_pk<PK_F32>(r, st);
  return run_chain_pk<PK_H16>(r, st);
}

template <typename T>
hipError_t pack(int N, int npairs, const void* Gl, const void* Gg, const void* Glb, const void* Ggb,
                int from_g, const ChainPlan& p, void* ws, bool h16, hipStream_t s) {
  unsigned* scal = reinterpret_cast<unsigned*>(at(ws, p.scal));
  if (h16) {
    // the chain's per-chunk maxima start from zero (a fill kernel, so the
    // sequence stays valid under stream capture)
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, scal, 2, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, scal + S_AMAX, 3, 0u);
  }
  const long long n = 2LL * N * N * npairs;
  hipLaunchKernelGGL(k_pack<T>, dim3(blocks(n, 256)), dim3(256), 0, s, N, npairs,
                     reinterpret_cast<const cplx*>(Gl), reinterpret_cast<const cplx*>(Gg),
                     reinterpret_cast<const cplx*>(Glb), reinterpret_cast<const cplx*>(Ggb), from_g,
                     reinterpret_cast<T*>(at(ws, p.gs)), reinterpret_cast<T*>(at(ws, p.gbs)),
                     h16 ? scal + S_GMAX : nullptr, h16 ? scal + S_GBMAX : nullptr);
  return hipGetLastError();
}

hipError_t prep_dispatch(int prec, int N, const double* v, const ChainPlan& p, void* ws, hipStream_t s,
                         bool packed = false) {
  StageTimer tm(4, s);
  if (packed) {
    if (prec == SB2_FP64) return prep_interaction<double, true>(N, v, p, ws, prec, s);
    if (prec == SB2_FP32) return prep_interaction<float, true>(N, v, p, ws, prec, s);
    return prep_interaction<_Float16, true>(N, v, p, ws, prec, s);
  }
  if (prec == SB2_FP64) return prep_interaction<double, false>(N, v, p, ws, prec, s);
  if (prec == SB2_FP32) return prep_interaction<float, false>(N, v, p, ws, prec, s);
  return prep_interaction<_Float16, false>(N, v, p, ws, prec, s);
}

hipError_t pack_dispatch(int prec, int N, int np, const void* Gl, const void* Gg, const void* Glb,
                         const void* Ggb, int from_g, const ChainPlan& p, void* ws, hipStream_t s) {
  StageTimer tm(6, s);
  if (prec == SB2_FP64) return pack<double>(N, np, Gl, Gg, Glb, Ggb, from_g, p, ws, false, s);
  return pack<float>(N, np, Gl, Gg, Glb, Ggb, from_g, p, ws, prec == SB2_SPLIT_FP16, s);
}

// Self-energies of `pairs` pairs (Gl[k], Gg[k]) -> S_less[k], S_great[k].
hipError_t sigma_pairs(int prec, int N, int pairs, const double* v, const void* Gl, const void* Gg,
                       const void* Glb, const void* Ggb, int from_g, cplx* S_less, cplx* S_great,
                       cplx* O_less, cplx* O_great, const ChainPlan& p, void* ws, hipStream_t s,
                       bool packed = false) {
  const size_t nn = (size_t)N * N;
  hipError_t e = prep_dispatch(prec, N, v, p, ws, s, packed);
  if (e != hipSuccess) return e;
  for (int k0 = 0; k0 < pairs; k0 += p.S) {
    const int np = pairs - k0 < p.S ? pairs - k0 : p.S;
    const size_t o = (size_t)k0 * nn * C128;
    e = pack_dispatch(prec, N, np, (const char*)Gl + o, (const char*)Gg + o,
                      Glb ? (const char*)Glb + o : nullptr, Ggb ? (const char*)Ggb + o : nullptr, from_g, p,
                      ws, s);
    if (e != hipSuccess) return e;
    e = run_chain(prec, N, 2 * np, p, ws, s);
    if (e != hipSuccess) return e;
    const long long nout = 2LL * np * N * N;
    StageTimer tm(6, s);
    hipLaunchKernelGGL(k_reduce_sigma, dim3(blocks(nout, 256)), dim3(256), 0, s, N, 2 * np, p.nz,
                       reinterpret_cast<const cplx*>(at(ws, p.part)), (i64)k0, S_less, S_great, O_less,
                       O_great);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// U[k] = exp(-i h (T-k) dt), k = 0..T-1: U_1 by scaling and squaring, then the
// powers U_1^m by doubling (P_{L+i} = P_L P_i), one batched product per level.
hipError_t propagators(int N, int T, const void* h, double dt, cplx* U, cplx* ex1, cplx* ex2, hipStream_t s) {
  const i64 nn = (i64)N * N;
  hipLaunchKernelGGL(k_expm, dim3(1), dim3(EXPM_THREADS), 0, s, N, reinterpret_cast<const cplx*>(h), 0.0, -dt,
                     U + (T - 1) * nn, ex1, ex2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int L = 1; L < T; L *= 2) {
    const int cnt = L < T - L ? L : T - L;
    GemmArgs g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = U + (T - L) * nn; g.sAm = N; g.sAk = 1; g.sAbh = 0;
    g.B = U + (T - 1) * nn; g.sBk = N; g.sBn = 1; g.sBbh = -nn;
    g.C = U + (T - L - 1) * nn; g.sCm = N; g.sCn = 1; g.sCbh = -nn;
    e = zgemm(g, cnt, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}


// Propagators and GKBA two-time functions for all past times (float64):
// U[k] = exp(-i h (T-k) dt), X = U rho, Y = rho U^dag and the four G's.
hipError_t gkba_history(int N, int T, const void* h, const void* rho_hist, double dt, cplx* U, cplx* X, cplx* Y,
                        cplx* Gl, cplx* Gg, cplx* Glb, cplx* Ggb, cplx* ex1, cplx* ex2, hipStream_t s) {
  StageTimer tm(5, s);
  const i64 nn = (i64)N * N;
  hipError_t e = propagators(N, T, h, dt, U, ex1, ex2, s);
  if (e != hipSuccess) return e;
  GemmArgs g = gdef();
  g.M = N; g.N = N; g.K = N;
  g.A = U; g.sAm = N; g.sAk = 1; g.sAbh = nn;
  g.B = rho_hist; g.sBk = N; g.sBn = 1; g.sBbh = nn;
  g.C = X; g.sCm = N; g.sCn = 1; g.sCbh = nn;
  if ((e = zgemm(g, T, s)) != hipSuccess) return e;
  g = gdef();
  g.M = N; g.N = N; g.K = N;
  g.A = rho_hist; g.sAm = N; g.sAk = 1; g.sAbh = nn;
  g.B = U; g.sBk = 1; g.sBn = N; g.sBbh = nn; g.conjB = 1;
  g.C = Y; g.sCm = N; g.sCn = 1; g.sCbh = nn;
  if ((e = zgemm(g, T, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_gkba, dim3(blocks((long long)T * nn, 256)), dim3(256), 0, s, N, T, U, X, Y, Gl, Gg, Glb, Ggb);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint of the collision integral (float64).  Per chunk of past times the
// forward chain R1..R4 is recomputed (A', B and C kept), the slices' Sigma
// cotangents are pulled back through R4..R1, and the cotangents of v (through
// both Vp and W_T), of G and of Gbar are accumulated; then the GKBA functions,
// the propagator powers and the exponential are differentiated in reverse.
// ---------------------------------------------------------------------------
struct BwdPlan {
  CollPlan f;          // forward history arrays (U, X, Y, G's, Sigma's)
  ChainPlan ch;        // chain buffers: W_T, Vp, Gs, GbT, A' (x1), B (x2), partials
  size_t c3, gc, gb, gss, gst, ggs, ggbs, part2, gwt, gvp, gsl, gsg, ggl, ggg, gglb, gggb, gu, gu1, scr;
  int nz2 = 1, kchunk2 = 16;
  size_t end;
};

constexpr size_t BWD_BUDGET = 24ull << 30;   // five chain-sized float64 buffers

BwdPlan bwd_plan(int N, int T) {
  BwdPlan b;
  b.f = coll_plan(N, T, SB2_FP64);
  const size_t n2 = (size_t)N * N, n3 = n2 * N, n4 = n3 * N;
  size_t S = BWD_BUDGET / (5 * 2 * n4 * C128);
  if (S < 1) S = 1;
  if (S > (size_t)T) S = T;
  const size_t smax = 65535 / (2 * (size_t)N);
  if (S > smax) S = smax;
  size_t o = b.f.end;
  b.ch = chain_plan(N, T, SB2_FP64, o, (int)S);
  o = b.ch.end;
  const size_t ns = 2 * S;
  // split-K of the three K = N^3 reductions: >= ~2048 workgroups (N x N
  // output tiles of the adjoint's products: 16 F rows, F as chosen by bwd_f,
  // by 64 columns)
  const int bm = 16 * (N <= 64 ? 4 : N <= 112 ? 7 : 8);
  const long long per_z = (long long)ns * ((N + bm - 1) / bm) * ((N + 63) / 64);
  long long nz = (2048 + per_z - 1) / per_z;
  long long kc = ((long long)n3 + nz - 1) / nz;
  kc = (kc + 15) / 16 * 16;
  b.kchunk2 = (int)kc;
  b.nz2 = (int)(((long long)n3 + kc - 1) / kc);
  const size_t hist = (size_t)T * n2 * C128;
  b.c3 = o; o += al(ns * n4 * C128);
  b.gc = o; o += al(ns * n4 * C128);
  b.gb = o; o += al(ns * n4 * C128);
  b.gss = o; o += al(ns * n2 * C128);
  b.gst = o; o += al(ns * n2 * C128);
  b.ggs = o; o += al(ns * n2 * C128);
  b.ggbs = o; o += al(ns * n2 * C128);
  b.part2 = o; o += al((size_t)b.nz2 * ns * n2 * C128);
  b.gwt = o; o += al(n3 * N * 8);
  b.gvp = o; o += al(n4 * 8);
  b.gsl = o; o += al(hist);
  b.gsg = o; o += al(hist);
  b.ggl = o; o += al(hist);
  b.ggg = o; o += al(hist);
  b.gglb = o; o += al(hist);
  b.gggb = o; o += al(hist);
  b.gu = o; o += al(hist);
  b.gu1 = o; o += al(n2 * C128);
  b.scr = o; o += al(6 * n2 * C128);
  b.end = o;
  return b;
}

// float64 GEMM configurations of the adjoint; F = 16-wide fragments per wave
// along the N-sized side (rows for zg_m*, columns for zg_n*), chosen from N so
// that the tile covers N with little padding (4 up to N = 64, 7 up to 112, 8)
template <int F>
hipError_t zg_m_f(GemmArgs g, int nb, hipStream_t s) { return launch_f<double, double, 1, 4, F, 1, true, true, false>(g, nb, s); }
template <int F>
hipError_t zg_n_f(GemmArgs g, int nb, hipStream_t s) { return launch_f<double, double, 4, 1, 1, F, true, true, false>(g, nb, s); }
template <int F>
hipError_t zg_n_rc_f(GemmArgs g, int nb, hipStream_t s) { return launch_f<double, double, 4, 1, 1, F, false, true, false>(g, nb, s); }
template <int F>
hipError_t zg_m_cr_f(GemmArgs g, int nb, hipStream_t s) { return launch_f<double, double, 1, 4, F, 1, true, false, false>(g, nb, s); }
template <int F>
hipError_t zg_m_k2_f(GemmArgs g, int nb, hipStream_t s) {
  constexpr int BM = 16 * F, BN = 64;
  if (g.kchunk <= 0) g.kchunk = g.K;
  g.tiles_m = (g.M + BM - 1) / BM;
  const int tiles_n = (g.N + BN - 1) / BN;
  const int nz = (g.K + g.kchunk - 1) / g.kchunk;
  dim3 grid(g.tiles_m * tiles_n, nb, nz);
  hipLaunchKernelGGL((k_gemm<double, double, 1, 4, F, 1, true, true, false, true>), grid, dim3(256), 0, s, g);
  return hipGetLastError();
}
inline int bwd_f(int N) { return N <= 64 ? 4 : N <= 112 ? 7 : 8; }
#define BWD_DISPATCH(name)                                              \
  hipError_t name(GemmArgs g, int nb, hipStream_t s, int N) {           \
    switch (bwd_f(N)) {                                                 \
      case 4: return name##_f<4>(g, nb, s);                             \
      case 7: return name##_f<7>(g, nb, s);                             \
      default: return name##_f<8>(g, nb, s);                            \
    }                                                                   \
  }
BWD_DISPATCH(zg_m)
BWD_DISPATCH(zg_n)
BWD_DISPATCH(zg_n_rc)
BWD_DISPATCH(zg_m_cr)
BWD_DISPATCH(zg_m_k2)
#undef BWD_DISPATCH

#define BW_TRY(expr)                          \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return e_;          \
  } while (0)

// ---------------------------------------------------------------------------
// Propagation with the collision integral accumulated over past times.  The
// step propagators compose, U(t_n, t_k) = P_n P_k^dag with P_n = U(t_n, t_0),
// so every GKBA function of past time k factors into P_n times a function of
// t_k alone (or that function times P_n^dag): G^<(t_n, t_k) = P_n a_k with
// a_k = i P_k^dag rho_k, G^>(t_n, t_k) = P_n b_k, G^<(t_k, t_n) = abar_k
// P_n^dag with abar_k = i rho_k P_k, G^>(t_k, t_n) = bbar_k P_n^dag.  In the
// self-energy (Eq. 13) the factors P_n attach to the t-side interaction
// v_irpn only (its legs n, p and r), so with the rotated interaction
//   vt(t_n)_{i r' p' n'} = sum_{n,p,r} v_irpn P_{n n'} P_{p p'} conj(P_{r r'})
// the collision integral (Eq. 9) becomes
//   I(t_n) = dt [ sum_{(n,p,r)} vt(t_n)[i][(n,p,r)] M_n[(n,p,r)][l] ] P_n^dag,
//   M_n = sum_{k<n} ( Ct^>_k abar_k - Ct^<_k bbar_k ),
// where Ct^<_k, Ct^>_k are the first three contractions of the chain (R1-R3)
// on (a_k, a_k, bbar_k) and (b_k, b_k, abar_k): they do not depend on t_n.
// One step therefore adds one past time to M and rotates v once, O(N^5)
// work, instead of running the chain over all n past times.
// ---------------------------------------------------------------------------
struct LinPlan {
  ChainPlan ch;                                   // chain buffers of one past time (two slices), float64
  size_t c3;                                      // Ct of the two slices
  size_t padj, x, y, gl, gg, glb, ggb;            // P_n^dag and the functions of the new past time
  size_t heff, ustep, I, T1, ex1, ex2, ptmp, ip;  // per-step N x N scratch
  size_t r1, r2;                                  // rotated interaction (N^4 complex each)
  size_t part;                                    // split-K partials of the last contraction
  int nz = 1, kchunk = 16;
  size_t end;
};

LinPlan lin_plan(int N) {
  LinPlan p;
  const size_t n2 = (size_t)N * N, n3 = n2 * N, n4 = n3 * N;
  const size_t m = al(n2 * C128);
  p.ch = chain_plan(N, 1, SB2_FP64, 0, 1);
  size_t o = p.ch.end;
  p.c3 = o; o += al(2 * n4 * C128);
  size_t* small[] = {&p.padj, &p.x, &p.y, &p.gl, &p.gg, &p.glb, &p.ggb, &p.heff, &p.ustep, &p.I, &p.T1,
                     &p.ex1, &p.ex2, &p.ptmp, &p.ip};
  for (size_t* q : small) { *q = o; o += m; }
  p.r1 = o; o += al(n4 * C128);
  p.r2 = o; o += al(n4 * C128);
  // split-K of the K = N^3 contraction: about 2048 workgroups of N x N output tiles
  const int bm = 16 * bwd_f(N);
  const long long per_z = (long long)((N + bm - 1) / bm) * ((N + 63) / 64);
  const long long nz = (2048 + per_z - 1) / per_z;
  long long kc = ((long long)n3 + nz - 1) / nz;
  kc = (kc + 15) / 16 * 16;
  p.kchunk = (int)kc;
  p.nz = (int)(((long long)n3 + kc - 1) / kc);
  p.part = o; o += al((size_t)p.nz * n2 * C128);
  p.end = o;
  return p;
}

hipError_t collision_backward(int N, int T, const double* v, const void* h, const void* rho, double dt,
                              const void* gI, double* gv, void* gh, void* grho, const BwdPlan& b, void* ws,
                              hipStream_t s) {
  const i64 n = N, n2 = n * n, n3 = n2 * n, n4 = n3 * n;
  auto P = [&](size_t off) { return reinterpret_cast<cplx*>(at(ws, off)); };
  cplx *U = P(b.f.U), *X = P(b.f.X), *Y = P(b.f.Y), *Gl = P(b.f.Gl), *Gg = P(b.f.Gg), *Glb = P(b.f.Glb),
       *Ggb = P(b.f.Ggb), *Sl = P(b.f.Sl), *Sg = P(b.f.Sg);
  cplx *gSl = P(b.gsl), *gSg = P(b.gsg), *gGl = P(b.ggl), *gGg = P(b.ggg), *gGlb = P(b.gglb), *gGgb = P(b.gggb),
       *gU = P(b.gu), *gU1 = P(b.gu1);
  const ChainPlan& ch = b.ch;
  const cplx* Gs = P(ch.gs);
  const cplx* GbT = P(ch.gbs);
  cplx *A1 = P(ch.x1), *B2 = P(ch.x2), *C3 = P(b.c3), *GC = P(b.gc), *GB = P(b.gb);
  cplx *gSs = P(b.gss), *gSt = P(b.gst), *gGs = P(b.ggs), *gGbs = P(b.ggbs), *part2 = P(b.part2);
  double* gWT = reinterpret_cast<double*>(at(ws, b.gwt));
  double* gVp = reinterpret_cast<double*>(at(ws, b.gvp));
  const double* WT = reinterpret_cast<const double*>(at(ws, ch.w));
  const double* Vp = reinterpret_cast<const double*>(at(ws, ch.vp));

  BW_TRY(gkba_history(N, T, h, rho, dt, U, X, Y, Gl, Gg, Glb, Ggb, P(b.f.ex1), P(b.f.ex2), s));
  BW_TRY(prep_dispatch(SB2_FP64, N, v, ch, ws, s));

  // Sigma cotangents: I = dt sum_k (Sigma^>_k Glb_k - Sigma^<_k Ggb_k)
  GemmArgs g = gdef();
  g.M = N; g.N = N; g.K = N;
  g.A = gI; g.sAm = N; g.sAk = 1;
  g.B = Glb; g.sBk = 1; g.sBn = N; g.sBbh = n2; g.conjB = 1;
  g.C = gSg; g.sCm = N; g.sCn = 1; g.sCbh = n2; g.alpha_re = dt;
  BW_TRY(zgemm(g, T, s));
  g.B = Ggb; g.C = gSl; g.alpha_re = -dt;
  BW_TRY(zgemm(g, T, s));

  const int S = ch.S;
  for (int k0 = 0; k0 < T; k0 += S) {
    const int np = T - k0 < S ? T - k0 : S;
    const int ns = 2 * np;
    const bool first = k0 == 0;
    const i64 ko = (i64)k0 * n2;
    // forward recompute of this chunk: A' (x1), B (x2), C (c3), Sigma
    BW_TRY(pack_dispatch(SB2_FP64, N, np, Gl + ko, Gg + ko, Glb + ko, Ggb + ko, 0, ch, ws, s));
    BW_TRY(run_chain(SB2_FP64, N, ns, ch, ws, s, C3));
    hipLaunchKernelGGL(k_reduce_sigma, dim3(blocks(2LL * np * n2, 256)), dim3(256), 0, s, N, ns, ch.nz,
                       reinterpret_cast<const cplx*>(at(ws, ch.part)), (i64)k0, Sl, Sg, (cplx*)nullptr,
                       (cplx*)nullptr);
    BW_TRY(hipGetLastError());
    // Gbar cotangents from the collision terms: gGlb = dt Sg^H gI, gGgb = -dt Sl^H gI
    g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = Sg + ko; g.sAm = 1; g.sAk = N; g.sAbh = n2; g.conjA = 1;
    g.B = gI; g.sBk = N; g.sBn = 1;
    g.C = gGlb + ko; g.sCm = N; g.sCn = 1; g.sCbh = n2; g.alpha_re = dt;
    BW_TRY(zgemm(g, np, s));
    g.A = Sl + ko; g.C = gGgb + ko; g.alpha_re = -dt;
    BW_TRY(zgemm(g, np, s));
    // slice cotangents
    hipLaunchKernelGGL(k_pack_gs, dim3(blocks(2LL * np * n2, 256)), dim3(256), 0, s, N, np, gSl + ko, gSg + ko, gSs,
                       gSt);
    BW_TRY(hipGetLastError());
    // R4 adjoint: gCt[b][(n,p)][j][r] = sum_i Vp[i][(n,p,r)] gS_b[i][j]
    g = gdef();
    g.M = (int)n3; g.N = N; g.K = N;
    g.A = Vp; g.sAm = 1; g.sAk = ch.KpV;
    g.B = gSs; g.sBk = N; g.sBn = 1; g.sBbh = n2;
    g.C = GC; g.Mlo = N; g.sCmh = n2; g.sCm = 1; g.sCn = N; g.sCbh = n4;
    BW_TRY(zg_n_rc(g, ns, s, N));
    // gVp[i][col] (+)= Re sum_{(b,j)} gS_b[i][j] conj(C_b[j][col])
    g = gdef();
    g.M = N; g.N = (int)n3; g.K = ns * N;
    g.A = gSt; g.sAm = (i64)ns * N; g.sAk = 1;
    g.B = C3; g.sBk = n3; g.sBn = 1; g.conjB = 1;
    g.C = gVp; g.sCm = n3; g.sCn = 1; g.out_real = 1; g.beta1 = first ? 0 : 1;
    BW_TRY(zg_m(g, 1, s, N));
    // R3 adjoint: gB[b][(n,p,j)][s] = sum_r gCt[b][(n,p,j)][r] conj(GbT[b][r][s])
    g = gdef();
    g.M = (int)n3; g.N = N; g.K = N;
    g.A = GC; g.sAm = N; g.sAk = 1; g.sAbh = n4;
    g.B = GbT; g.sBk = N; g.sBn = 1; g.sBbh = n2; g.conjB = 1;
    g.C = GB; g.sCm = N; g.sCn = 1; g.sCbh = n4;
    BW_TRY(zg_n(g, ns, s, N));
    // gGbar_b[s][r] = sum_{(n,p,j)} conj(B_b[(n,p,j)][s]) gCt_b[(n,p,j)][r]   (split-K)
    g = gdef();
    g.M = N; g.N = N; g.K = (int)n3; g.kchunk = b.kchunk2;
    g.A = B2; g.sAm = 1; g.sAk = N; g.sAbh = n4; g.conjA = 1;
    g.B = GC; g.sBk = N; g.sBn = 1; g.sBbh = n4;
    g.C = part2; g.sCm = N; g.sCn = 1; g.sCbh = n2; g.sCz = (i64)ns * n2;
    BW_TRY(zg_m(g, ns, s, N));
    hipLaunchKernelGGL(k_sum_partials, dim3(blocks((long long)ns * n2, 256)), dim3(256), 0, s, (i64)ns * n2,
                       b.nz2, part2, gGbs, 0);
    BW_TRY(hipGetLastError());
    // R2 adjoint: gA'[b][n][x][q] = sum_p gB[b][n][p][x] conj(G_b[p][q])   (into GC)
    g = gdef();
    g.M = (int)n2; g.N = N; g.K = N; g.nbl = N;
    g.A = GB; g.sAm = 1; g.sAk = n2; g.sAbh = n4; g.sAbl = n3;
    g.B = Gs; g.sBk = N; g.sBn = 1; g.sBbh = n2; g.sBbl = 0; g.conjB = 1;
    g.C = GC; g.sCm = N; g.sCn = 1; g.sCbh = n4; g.sCbl = n3;
    BW_TRY(zg_n(g, ns * N, s, N));
    // gG_b[p][q] = sum_{(n,x)} gB[b][n][p][x] conj(A'[b][n][x][q])   (second G slot, split-K)
    g = gdef();
    g.M = N; g.N = N; g.K = (int)n3; g.kchunk = b.kchunk2; g.Klo = (int)n2;
    g.A = GB; g.sAm = n2; g.sAk = 1; g.sAkh = n3; g.sAbh = n4;
    g.B = A1; g.sBk = N; g.sBkh = n3; g.sBn = 1; g.sBbh = n4; g.conjB = 1;
    g.C = part2; g.sCm = N; g.sCn = 1; g.sCbh = n2; g.sCz = (i64)ns * n2;
    BW_TRY(zg_m_k2(g, ns, s, N));
    hipLaunchKernelGGL(k_sum_partials, dim3(blocks((long long)ns * n2, 256)), dim3(256), 0, s, (i64)ns * n2,
                       b.nz2, part2, gGs, 0);
    BW_TRY(hipGetLastError());
    // gG_b[n][m] += sum_col gA'[b][n][col] W_T[col][m]   (first G slot, split-K)
    g = gdef();
    g.M = N; g.N = N; g.K = (int)n3; g.kchunk = b.kchunk2;
    g.A = GC; g.sAm = n3; g.sAk = 1; g.sAbh = n4;
    g.B = WT; g.sBk = ch.KpW; g.sBn = 1;
    g.C = part2; g.sCm = N; g.sCn = 1; g.sCbh = n2; g.sCz = (i64)ns * n2;
    BW_TRY(zg_m_cr(g, ns, s, N));
    hipLaunchKernelGGL(k_sum_partials, dim3(blocks((long long)ns * n2, 256)), dim3(256), 0, s, (i64)ns * n2,
                       b.nz2, part2, gGs, 1);
    BW_TRY(hipGetLastError());
    // gWT[col][m] (+)= Re sum_{(b,n)} gA'[(b,n)][col] conj(G[(b,n)][m])
    g = gdef();
    g.M = (int)n3; g.N = N; g.K = ns * N;
    g.A = GC; g.sAm = 1; g.sAk = n3;
    g.B = Gs; g.sBk = N; g.sBn = 1; g.conjB = 1;
    g.C = gWT; g.sCm = N; g.sCn = 1; g.out_real = 1; g.beta1 = first ? 0 : 1;
    BW_TRY(zg_n(g, 1, s, N));
    hipLaunchKernelGGL(k_scatter_gg, dim3(blocks((long long)np * n2, 256)), dim3(256), 0, s, N, np, gGs, gGbs,
                       gGl + ko, gGg + ko, gGlb + ko, gGgb + ko);
    BW_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_assemble_gv, dim3(blocks(n4, 256)), dim3(256), 0, s, N, gWT, gVp, gv);
  BW_TRY(hipGetLastError());

  // GKBA adjoint: gX = -i(gGl + gGg), gY = -i(gGlb + gGgb), gU = i gGg - i gGgb^dag  (gX, gY reuse X, Y)
  hipLaunchKernelGGL(k_gkba_adj, dim3(blocks((long long)T * n2, 256)), dim3(256), 0, s, N, T, gGl, gGg, gGlb, gGgb,
                     X, Y, gU);
  BW_TRY(hipGetLastError());
  cplx* gX = X;
  cplx* gY = Y;
  // gU += gX rho^H + gY^H rho
  g = gdef();
  g.M = N; g.N = N; g.K = N;
  g.A = gX; g.sAm = N; g.sAk = 1; g.sAbh = n2;
  g.B = rho; g.sBk = 1; g.sBn = N; g.sBbh = n2; g.conjB = 1;
  g.C = gU; g.sCm = N; g.sCn = 1; g.sCbh = n2; g.beta1 = 1;
  BW_TRY(zgemm(g, T, s));
  g = gdef();
  g.M = N; g.N = N; g.K = N;
  g.A = gY; g.sAm = 1; g.sAk = N; g.sAbh = n2; g.conjA = 1;
  g.B = rho; g.sBk = N; g.sBn = 1; g.sBbh = n2;
  g.C = gU; g.sCm = N; g.sCn = 1; g.sCbh = n2; g.beta1 = 1;
  BW_TRY(zgemm(g, T, s));
  // grho = U^H gX + gY U
  g = gdef();
  g.M = N; g.N = N; g.K = N;
  g.A = U; g.sAm = 1; g.sAk = N; g.sAbh = n2; g.conjA = 1;
  g.B = gX; g.sBk = N; g.sBn = 1; g.sBbh = n2;
  g.C = grho; g.sCm = N; g.sCn = 1; g.sCbh = n2;
  BW_TRY(zgemm(g, T, s));
  g = gdef();
  g.M = N; g.N = N; g.K = N;
  g.A = gY; g.sAm = N; g.sAk = 1; g.sAbh = n2;
  g.B = U; g.sBk = N; g.sBn = 1; g.sBbh = n2;
  g.C = grho; g.sCm = N; g.sCn = 1; g.sCbh = n2; g.beta1 = 1;
  BW_TRY(zgemm(g, T, s));

  // powers: U[k] = P_m, m = T - k, P_m = U1 P_{m-1}.  Reverse sweep m = T..2:
  //   gU1 += gP_m P_{m-1}^H,  gP_{m-1} += U1^H gP_m;  finally gU1 += gP_1.
  const cplx* U1 = U + (i64)(T - 1) * n2;
  hipLaunchKernelGGL(k_copy, dim3(blocks(n2, 256)), dim3(256), 0, s, (i64)n2, gU + (i64)(T - 1) * n2, gU1);
  BW_TRY(hipGetLastError());
  for (int m = T; m >= 2; --m) {
    const i64 km = (i64)(T - m) * n2, km1 = (i64)(T - m + 1) * n2;
    g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = gU + km; g.sAm = N; g.sAk = 1;
    g.B = U + km1; g.sBk = 1; g.sBn = N; g.conjB = 1;
    g.C = gU1; g.sCm = N; g.sCn = 1; g.beta1 = 1;
    BW_TRY(zgemm(g, 1, s));
    if (m - 1 >= 2) {
      g = gdef();
      g.M = N; g.N = N; g.K = N;
      g.A = U1; g.sAm = 1; g.sAk = N; g.conjA = 1;
      g.B = gU + km; g.sBk = N; g.sBn = 1;
      g.C = gU + km1; g.sCm = N; g.sCn = 1; g.beta1 = 1;
      BW_TRY(zgemm(g, 1, s));
    }
  }
  // gP_1 for m = 1 is gU[T-1] plus the chain's contributions accumulated above (when T >= 2 the
  // m = 2 step folded U1^H gP_2 into gU[T-1] only if it was applied; do it here instead)
  if (T >= 2) {
    g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = U1; g.sAm = 1; g.sAk = N; g.conjA = 1;
    g.B = gU + (i64)(T - 2) * n2; g.sBk = N; g.sBn = 1;
    g.C = gU1; g.sCm = N; g.sCn = 1; g.beta1 = 1;
    BW_TRY(zgemm(g, 1, s));
  }
  // U1 = exp(A), A = -i dt h:  gA = L_exp(A^H, gU1),  gh = i dt gA
  hipLaunchKernelGGL(k_expm_frechet, dim3(1), dim3(EXPM_THREADS), 0, s, N, reinterpret_cast<const cplx*>(h), 1, 0.0,
                     dt, gU1, reinterpret_cast<cplx*>(gh), P(b.scr));
  BW_TRY(hipGetLastError());
  // gh <- i dt gA  (scale in place)
  g = gdef();
  (void)g;
  hipLaunchKernelGGL(k_scale_c, dim3(blocks(n2, 256)), dim3(256), 0, s, (i64)n2, reinterpret_cast<cplx*>(gh), 0.0, dt);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched evaluation of several systems.  All systems advance in R common
// rounds (system b takes S_b = ceil(T_b / R) past times per round, R as small
// as the intermediate budget allows); in every round each chain stage is ONE
// grouped launch over all systems that still have past times left.  The
// per-system set-up (interaction layout, propagators, GKBA functions) and the
// collision sums are per-system launches around the rounds.
// ---------------------------------------------------------------------------
constexpr size_t BATCH_BUDGET = 96ull << 30;

struct BatchPlan {
  int rounds = 1;
  bool chunked = false;     // members use the fused split-float16 chain
  std::vector<CollPlan> cp;
  std::vector<size_t> base;
  std::vector<double> work;   // algorithmic work of one round of each member (S_b N_b^5)
  size_t refs = 0;     // device ChainRefs table
  size_t end = 0;
};

// Past times of member b per round when the longest member takes R rounds:
// ceil(T_b / R), but at least enough for 2 S_b N_b >= 768 rows of the first
// contraction, so that small systems keep full tiles (they then finish in
// fewer rounds), and at most what one launch's grid.y holds.
size_t batch_chunk(const sb2_system& q, int R) {
  size_t S = ((size_t)q.T + R - 1) / R;
  const size_t smin = (384 + (size_t)q.N - 1) / q.N;
  if (S < smin) S = smin;
  if (S > (size_t)q.T) S = q.T;
  return S;
}

BatchPlan batch_plan(int nsys, const sb2_system* sys, int prec) {
  BatchPlan bp;
  // the fused split-float16 path (n-chunked layouts) when every member can take it
  bool chunked = prec == SB2_SPLIT_FP16;
  for (int b = 0; b < nsys; ++b)
    if (sys[b].N > R23_MAX_N || tune_of(sys[b].N, prec).r23 <= 0) chunked = false;
  bp.chunked = chunked;
  const size_t bb = bulk_bytes(prec);
  int R = 1;
  for (;; ++R) {
    size_t tot = 0;
    bool fits_grid = true;
    for (int b = 0; b < nsys; ++b) {
      const size_t n4 = (size_t)sys[b].N * sys[b].N * sys[b].N * sys[b].N;
      const size_t S = batch_chunk(sys[b], R);
      tot += S * 2 * 2 * n4 * 2 * bb;
      if (S > 65535 / (2 * (size_t)sys[b].N)) fits_grid = false;
    }
    if ((tot <= BATCH_BUDGET && fits_grid) || R >= SB2_MAX_T) break;
  }
  bp.rounds = R;
  double wsum = 0.0;
  for (int b = 0; b < nsys; ++b) {
    const double n = sys[b].N;
    bp.work.push_back((double)batch_chunk(sys[b], R) * n * n * n * n * n);
    wsum += bp.work.back();
  }
  size_t o = 0;
  bp.refs = o;
  o += al(sizeof(ChainRefs) * MAX_GROUP);
  for (int b = 0; b < nsys; ++b) {
    const int S = (int)batch_chunk(sys[b], R);
    bp.cp.push_back(coll_plan(sys[b].N, sys[b].T, prec, S, bp.work[b] / wsum, chunked));
    bp.base.push_back(o);
    o += bp.cp.back().end;
  }
  bp.end = o;
  return bp;
}

// share[i]: member i's part of the launch's work; the workgroup target of the
// single-slab stages is divided among the members in that proportion.
template <int PK, int STAGE, int FSN>
hipError_t launch_group_fs(const std::vector<ChainRefs>& refs, const std::vector<double>& share,
                           const ChainRefs* d_refs, hipStream_t st) {
  GroupTable t;
  t.count = (int)refs.size();
  long long off = 0;
  for (int i = 0; i < t.count; ++i) {
    t.off[i] = off;
    const double want = tune_of(refs[i].N, refs[i].prec).persist * share[i];
    t.persist[i] = want < 1.0 ? 1 : (int)want;
    int nbatch;
    StreamArgs g = stage_args(STAGE, refs[i], nbatch);
    off += stage_geom<PK, STAGE, FSN>(g, nbatch, t.persist[i]).blocks();
  }
  t.off[t.count] = off;
  if (off <= 0) return hipSuccess;
  StageTimer tm(STAGE, st);
  hipLaunchKernelGGL((k_stage_group<PK, STAGE, FSN>), dim3((unsigned)off), dim3(64 * StageCfg<PK, STAGE>::NW), 0,
                     st, d_refs, t);
  return hipGetLastError();
}

// the members of a group share ceil(N/16), hence the tile height of stages 1-3
template <int PK, int STAGE>
hipError_t launch_group(const std::vector<ChainRefs>& refs, const std::vector<double>& share, const ChainRefs* d_refs,
                        hipStream_t st) {
  int nmax = 1;
  for (const ChainRefs& r : refs) nmax = std::max(nmax, r.N);
  if constexpr (STAGE == 0) {
    return launch_group_fs<PK, 0, 0>(refs, share, d_refs, st);
  } else {
    switch (stage_fs(nmax)) {
      case 2: return launch_group_fs<PK, STAGE, 2>(refs, share, d_refs, st);
      case 4: return launch_group_fs<PK, STAGE, 4>(refs, share, d_refs, st);
      case 6: return launch_group_fs<PK, STAGE, 6>(refs, share, d_refs, st);
      case 7: return launch_group_fs<PK, STAGE, 7>(refs, share, d_refs, st);
      default: return launch_group_fs<PK, STAGE, 8>(refs, share, d_refs, st);
    }
  }
}

template <int PK>
hipError_t group_chain(const std::vector<ChainRefs>& refs, const std::vector<double>& sh, const ChainRefs* d,
                       hipStream_t st) {
  hipError_t e;
  if ((e = launch_group<PK, 0>(refs, sh, d, st)) != hipSuccess) return e;
  if ((e = launch_group<PK, 1>(refs, sh, d, st)) != hipSuccess) return e;
  if ((e = launch_group<PK, 2>(refs, sh, d, st)) != hipSuccess) return e;
  return launch_group<PK, 3>(refs, sh, d, st);
}

template <int NT>
hipError_t launch_bucket(const ChainRefs* d, const SubGroup& t23, const SubGroup& t4, hipStream_t st) {
  hipError_t e;
  {
    StageTimer tm(1, st);
    hipLaunchKernelGGL((k_r23_group<NT>), dim3((unsigned)t23.off[t23.count]), dim3(R23Cfg<NT>::NTH), 0, st, d, t23);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  StageTimer tm(3, st);
  hipLaunchKernelGGL((k_r4_group<NT>), dim3((unsigned)t4.off[t4.count]), dim3(R4_THREADS), 0, st, d, t4);
  return hipGetLastError();
}

// One round of the n-chunked split-float16 chain over all members: the first
// contraction as one grouped launch, then per 16-wide bucket of N one launch
// of the fused second+third and one of the last contraction.  Each bucket's
// fused launch gets about the single-system workgroup count, divided among
// its members by work.
hipError_t group_chain_h16(const std::vector<ChainRefs>& refs, const std::vector<double>& share, const ChainRefs* d,
                           hipStream_t st) {
  hipError_t e;
  if ((e = launch_group<PK_H16, 0>(refs, share, d, st)) != hipSuccess) return e;
  for (int nt = 1; nt <= 7; ++nt) {
    SubGroup t23, t4;
    t23.count = t4.count = 0;
    double wsum = 0.0;
    for (size_t i = 0; i < refs.size(); ++i)
      if ((refs[i].N + 15) / 16 == nt) wsum += share[i];
    long long o23 = 0, o4 = 0;
    for (size_t i = 0; i < refs.size(); ++i) {
      if ((refs[i].N + 15) / 16 != nt) continue;
      const long long ntask = (long long)refs[i].ns * refs[i].N * refs[i].N;
      // grouped members are small systems: a generous workgroup count (more
      // for fewer waves per workgroup) keeps the chip filled
      long long nwg = (long long)(4.0 * r23_wgs(refs[i].N, refs[i].prec) * 7 / nt * share[i] / wsum + 0.5);
      if (nwg < 1) nwg = 1;
      if (nwg > ntask) nwg = ntask;
      t23.idx[t23.count] = t4.idx[t4.count] = (int)i;
      t23.off[t23.count++] = o23;
      t4.off[t4.count++] = o4;
      o23 += nwg;
      o4 += (long long)r4_tiles(r4_args(refs[i])) * refs[i].N;
    }
    if (t23.count == 0) continue;
    t23.off[t23.count] = o23;
    t4.off[t4.count] = o4;
    switch (nt) {
      case 1: e = launch_bucket<1>(d, t23, t4, st); break;
      case 2: e = launch_bucket<2>(d, t23, t4, st); break;
      case 3: e = launch_bucket<3>(d, t23, t4, st); break;
      case 4: e = launch_bucket<4>(d, t23, t4, st); break;
      case 5: e = launch_bucket<5>(d, t23, t4, st); break;
      case 6: e = launch_bucket<6>(d, t23, t4, st); break;
      default: e = launch_bucket<7>(d, t23, t4, st); break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// A system with at least SOLO_FLOPS of contraction work (48 T N^5) fills the
// chip with its own launches, and grouping it only shrinks its chunks: it
// runs as a single-system chain.  Smaller systems share grouped launches.
constexpr double SOLO_FLOPS = 1e12;
inline bool batch_solo(const sb2_system& q) {
  const double n = q.N;
  return 48.0 * q.T * n * n * n * n * n >= SOLO_FLOPS;
}

// Systems grouped by ceil(N/16), in order of first appearance (solo systems excluded).
std::vector<std::vector<sb2_system>> size_buckets(int nsys, const sb2_system* sys) {
  std::vector<std::vector<sb2_system>> out;
  std::vector<int> key;
  for (int b = 0; b < nsys; ++b) {
    if (batch_solo(sys[b])) continue;
    const int k = (sys[b].N + 15) / 16;
    size_t i = 0;
    while (i < key.size() && key[i] != k) ++i;
    if (i == key.size()) {
      key.push_back(k);
      out.emplace_back();
    }
    out[i].push_back(sys[b]);
  }
  return out;
}

hipError_t collision_batched(int nsys, const sb2_system* sys, int prec, const BatchPlan& bp, void* ws,
                             hipStream_t s) {
  hipError_t e;
  std::vector<char*> wsb(nsys);
  for (int b = 0; b < nsys; ++b) wsb[b] = reinterpret_cast<char*>(ws) + bp.base[b];
  // per-system set-up: interaction layouts, propagators and GKBA functions
  for (int b = 0; b < nsys; ++b) {
    const CollPlan& c = bp.cp[b];
    void* w = wsb[b];
    auto P = [&](size_t off) { return reinterpret_cast<cplx*>(at(w, off)); };
    if ((e = gkba_history(sys[b].N, sys[b].T, sys[b].h, sys[b].rho_hist, sys[b].dt, P(c.U), P(c.X), P(c.Y), P(c.Gl),
                          P(c.Gg), P(c.Glb), P(c.Ggb), P(c.ex1), P(c.ex2), s)) != hipSuccess)
      return e;
    if ((e = prep_dispatch(prec, sys[b].N, sys[b].v, c.ch, w, s)) != hipSuccess) return e;
  }
  ChainRefs* d_refs = reinterpret_cast<ChainRefs*>(at(ws, bp.refs));
  for (int r = 0; r < bp.rounds; ++r) {
    std::vector<ChainRefs> refs;
    std::vector<int> who, kk0, nps;
    std::vector<double> share;
    double wsum = 0.0;
    for (int b = 0; b < nsys; ++b) {
      const CollPlan& c = bp.cp[b];
      const int k0 = r * c.ch.S;
      if (k0 >= sys[b].T) continue;
      const int np = sys[b].T - k0 < c.ch.S ? sys[b].T - k0 : c.ch.S;
      const int N = sys[b].N;
      const size_t o = (size_t)k0 * N * N * C128;
      void* w = wsb[b];
      if ((e = pack_dispatch(prec, N, np, at(w, c.Gl + o), at(w, c.Gg + o), at(w, c.Glb + o), at(w, c.Ggb + o), 0,
                             c.ch, w, s)) != hipSuccess)
        return e;
      refs.push_back(chain_refs(prec, N, 2 * np, c.ch, w, nullptr));
      who.push_back(b);
      kk0.push_back(k0);
      nps.push_back(np);
      share.push_back(bp.work[b] * np / c.ch.S);
      wsum += share.back();
    }
    if (refs.empty()) break;
    for (double& x : share) x /= wsum;
    for (size_t i0 = 0; i0 < refs.size(); i0 += REFS_PER_WRITE) {
      RefsChunk ck;
      ck.count = (int)std::min(refs.size() - i0, (size_t)REFS_PER_WRITE);
      for (int i = 0; i < ck.count; ++i) ck.r[i] = refs[i0 + i];
      hipLaunchKernelGGL(k_write_refs, dim3(1), dim3(64), 0, s, d_refs + i0, ck);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (prec == SB2_FP64) e = group_chain<PK_F64>(refs, share, d_refs, s);
    else if (prec == SB2_FP32) e = group_chain<PK_F32>(refs, share, d_refs, s);
    else if (bp.chunked) e = group_chain_h16(refs, share, d_refs, s);
    else e = group_chain<PK_H16>(refs, share, d_refs, s);
    if (e != hipSuccess) return e;
    for (size_t i = 0; i < refs.size(); ++i) {
      const int b = who[i];
      const CollPlan& c = bp.cp[b];
      const int N = sys[b].N;
      void* w = wsb[b];
      StageTimer tm(6, s);
      hipLaunchKernelGGL(k_reduce_sigma, dim3(blocks(2LL * nps[i] * N * N, 256)), dim3(256), 0, s, N, 2 * nps[i],
                         c.ch.nz, reinterpret_cast<const cplx*>(at(w, c.ch.part)), (i64)kk0[i],
                         reinterpret_cast<cplx*>(at(w, c.Sl)), reinterpret_cast<cplx*>(at(w, c.Sg)), (cplx*)nullptr,
                         (cplx*)nullptr);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  // collision sums per system
  for (int b = 0; b < nsys; ++b) {
    const CollPlan& c = bp.cp[b];
    const int N = sys[b].N, T = sys[b].T;
    const i64 nn = (i64)N * N;
    void* w = wsb[b];
    auto P = [&](size_t off) { return reinterpret_cast<cplx*>(at(w, off)); };
    StageTimer tm(7, s);
    GemmArgs g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = P(c.Sg); g.sAm = N; g.sAk = 1; g.sAbh = nn;
    g.B = P(c.Glb); g.sBk = N; g.sBn = 1; g.sBbh = nn;
    g.C = P(c.terms); g.sCm = N; g.sCn = 1; g.sCbh = nn;
    if ((e = zgemm(g, T, s)) != hipSuccess) return e;
    g.A = P(c.Sl); g.B = P(c.Ggb); g.alpha_re = -1.0; g.beta1 = 1;
    if ((e = zgemm(g, T, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_terms, dim3(blocks(nn, 256)), dim3(256), 0, s, N, T, P(c.terms), sys[b].dt,
                       reinterpret_cast<cplx*>(sys[b].I_out), (const double*)nullptr, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* sb2_version(void) { return "sb2 0.1 (gfx950)"; }

int sb2_profile_enable(int on) {
  g_prof.on = on != 0;
  g_prof.recs.clear();
  g_prof.used = 0;
  return SB2_OK;
}

int sb2_profile_read(double* ms, int* launches, int nslots) {
  if (!ms || !launches || nslots < 1) return SB2_EINVAL;
  for (int i = 0; i < nslots; ++i) { ms[i] = 0.0; launches[i] = 0; }
  for (const ProfRec& r : g_prof.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return SB2_EHIP;
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return SB2_EHIP;
    if (r.slot < nslots) { ms[r.slot] += t; launches[r.slot] += 1; }
  }
  g_prof.recs.clear();
  g_prof.used = 0;
  return SB2_OK;
}

const char* sb2_status_string(int status) {
  switch (status) {
    case SB2_OK: return "ok";
    case SB2_EINVAL: return "invalid argument (null pointer, non-finite or non-positive dt, or unknown enum)";
    case SB2_ESHAPE: return "size out of range (N, T or batch count)";
    case SB2_EWORKSPACE: return "workspace smaller than sb2_workspace_size()";
    case SB2_EHIP: return "HIP runtime error while enqueueing work";
    case SB2_EUNSUPPORTED: return "precision not supported by this entry point (SB2_SPLIT_BF16 is not built)";
    case SB2_ECHECK:
      return "input check failed (SB2_CHECK=1): a non-finite input, or h or a density matrix not Hermitian";
    case SB2_ESCRATCH:
      return "problem needs more scratch memory than the static buffer of sb2_collision_noalloc "
             "(SB2_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown status";
  }
}

size_t sb2_workspace_size(int op, int N, int T, int prec) {
  if (N < 1 || N > SB2_MAX_N || !prec_ok(prec)) return 0;
  switch (op) {
    case SB2_OP_SIGMA:
      if (T < 1) return 0;
      return chain_plan(N, T, prec, 0).end;
    case SB2_OP_COLLISION:
      if (T < 1 || T > SB2_MAX_T) return 0;
      return coll_plan(N, T, prec).end;
    case SB2_OP_RHO_STEP:
      return rho_plan(N);
    case SB2_OP_COLLISION_BACKWARD:
      if (T < 1 || T > SB2_MAX_T || prec != SB2_FP64) return 0;
      return bwd_plan(N, T).end;
    case SB2_OP_AUTOTUNE:
      if (T < 1 || T > SB2_MAX_T) return 0;
      return tune_bytes(N, T, prec);
    case SB2_OP_PROPAGATE:
      if (T < 1 || T > SB2_MAX_T) return 0;
      return prop_plan(N, T, prec).end;
    case SB2_OP_COLLISION_DIAGONAL:
      if (T < 1 || T > SB2_MAX_T) return 0;
      return vert_plan(N, T, SB2_VERTEX_DIAGONAL).end;
    case SB2_OP_COLLISION_SYMMETRIC:
      if (T < 1 || T > SB2_MAX_T) return 0;
      return vert_plan(N, T, SB2_VERTEX_SYMMETRIC).end;
    case SB2_OP_PROPAGATE_DIAGONAL:
      if (T < 1 || T > SB2_MAX_T) return 0;
      return prop_plan(N, T, SB2_FP64, SB2_VERTEX_DIAGONAL).end;
    case SB2_OP_PROPAGATE_SYMMETRIC:
      if (T < 1 || T > SB2_MAX_T) return 0;
      return prop_plan(N, T, SB2_FP64, SB2_VERTEX_SYMMETRIC).end;
    case SB2_OP_PROPAGATE_LINEAR:
      return lin_plan(N).end;
    default:
      return 0;
  }
}

int sb2_sigma(int N, int B, const double* v, const void* Gl, const void* Gg, void* Sl, void* Sg, int prec,
              void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || N > SB2_MAX_N || B < 1) return SB2_ESHAPE;
  if (!v || !Gl || !Gg || !Sl || !Sg || !ws) return SB2_EINVAL;
  SB2_PREC(prec);
  const ChainPlan p = chain_plan(N, B, prec, 0);
  if (ws_bytes < p.end) return SB2_EWORKSPACE;
  SB2_ENTRY();
  SB2_CHECKS(ws, N, {2, v, (i64)N * N * N * N}, {1, Gl, (i64)B * N * N}, {1, Gg, (i64)B * N * N});
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = sigma_pairs(prec, N, B, v, Gl, Gg, nullptr, nullptr, 1, reinterpret_cast<cplx*>(Sl),
                             reinterpret_cast<cplx*>(Sg), nullptr, nullptr, p, ws, s);
  return e == hipSuccess ? SB2_OK : SB2_EHIP;
}

// I = dt sum_k [Sigma^>_k G^<(t_k,t) - Sigma^<_k G^>(t_k,t)] (Eq. 9), float64.
hipError_t collision_terms(int N, int T, const cplx* Sl, const cplx* Sg, const cplx* Glb, const cplx* Ggb,
                           cplx* terms, double dt, cplx* I_out, hipStream_t s, const double* lam = nullptr,
                           int now = 0) {
  const i64 nn = (i64)N * N;
  StageTimer tm(7, s);
  GemmArgs g = gdef();
  g.M = N; g.N = N; g.K = N;
  g.A = Sg; g.sAm = N; g.sAk = 1; g.sAbh = nn;
  g.B = Glb; g.sBk = N; g.sBn = 1; g.sBbh = nn;
  g.C = terms; g.sCm = N; g.sCn = 1; g.sCbh = nn;
  hipError_t e;
  if ((e = zgemm(g, T, s)) != hipSuccess) return e;
  g.A = Sl; g.B = Ggb; g.alpha_re = -1.0; g.beta1 = 1;
  if ((e = zgemm(g, T, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_terms, dim3(blocks(nn, 256)), dim3(256), 0, s, N, T, terms, dt, I_out, lam, now);
  return hipGetLastError();
}

// Collision integral from given propagators U[k] = U(t, t_k), k < T (Eq. 10
// with Eq. 11's propagators supplied): X_k = U_k rho_k, Y_k = rho_k U_k^dag,
// the four GKBA functions, the self-energy chain and the k-sum.
hipError_t collision_core(int N, int T, const double* v, const cplx* U, const void* rho_hist, double dt,
                          cplx* I_out, cplx* Sigma_out, int prec, const CollPlan& c, void* ws, hipStream_t s,
                          bool packed = false, const double* lam = nullptr, int now = 0) {
  const i64 nn = (i64)N * N;
  cplx* X = reinterpret_cast<cplx*>(at(ws, c.X));
  cplx* Y = reinterpret_cast<cplx*>(at(ws, c.Y));
  cplx* Gl = reinterpret_cast<cplx*>(at(ws, c.Gl));
  cplx* Gg = reinterpret_cast<cplx*>(at(ws, c.Gg));
  cplx* Glb = reinterpret_cast<cplx*>(at(ws, c.Glb));
  cplx* Ggb = reinterpret_cast<cplx*>(at(ws, c.Ggb));
  cplx* Sl = reinterpret_cast<cplx*>(at(ws, c.Sl));
  cplx* Sg = reinterpret_cast<cplx*>(at(ws, c.Sg));
  cplx* terms = reinterpret_cast<cplx*>(at(ws, c.terms));
  hipError_t e;
  GemmArgs g;
  {
    StageTimer tm(5, s);
    g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = U; g.sAm = N; g.sAk = 1; g.sAbh = nn;
    g.B = rho_hist; g.sBk = N; g.sBn = 1; g.sBbh = nn;
    g.C = X; g.sCm = N; g.sCn = 1; g.sCbh = nn;
    if ((e = zgemm(g, T, s)) != hipSuccess) return e;
    g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = rho_hist; g.sAm = N; g.sAk = 1; g.sAbh = nn;
    g.B = U; g.sBk = 1; g.sBn = N; g.sBbh = nn; g.conjB = 1;
    g.C = Y; g.sCm = N; g.sCn = 1; g.sCbh = nn;
    if ((e = zgemm(g, T, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gkba, dim3(blocks((long long)T * nn, 256)), dim3(256), 0, s, N, T, U, X, Y, Gl, Gg, Glb,
                       Ggb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }

  cplx* Ol = Sigma_out;
  cplx* Og = Sigma_out ? Ol + (i64)T * nn : nullptr;
  if ((e = sigma_pairs(prec, N, T, v, Gl, Gg, Glb, Ggb, 0, Sl, Sg, Ol, Og, c.ch, ws, s, packed)) != hipSuccess)
    return e;
  return collision_terms(N, T, Sl, Sg, Glb, Ggb, terms, dt, I_out, s, lam, now);
}

int sb2_collision(int N, int T, const double* v, const void* h, const void* rho_hist, double dt, void* I_out,
                  void* Sigma_out, int prec, void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || N > SB2_MAX_N || T < 1 || T > SB2_MAX_T) return SB2_ESHAPE;
  if (!v || !h || !rho_hist || !I_out || !ws || !finite_pos(dt)) return SB2_EINVAL;
  SB2_PREC(prec);
  const CollPlan c = coll_plan(N, T, prec);
  if (ws_bytes < c.end) return SB2_EWORKSPACE;
  SB2_ENTRY();
  SB2_CHECKS(ws, N, {2, v, (i64)N * N * N * N}, {0, h, 1}, {0, rho_hist, T});
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  cplx* U = reinterpret_cast<cplx*>(at(ws, c.U));
  {
    StageTimer tm(5, s);
    SB2_TRY(propagators(N, T, h, dt, U, reinterpret_cast<cplx*>(at(ws, c.ex1)),
                        reinterpret_cast<cplx*>(at(ws, c.ex2)), s));
  }
  SB2_TRY(collision_core(N, T, v, U, rho_hist, dt, reinterpret_cast<cplx*>(I_out),
                         reinterpret_cast<cplx*>(Sigma_out), prec, c, ws, s));
  return SB2_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free variant of sb2_collision: its scratch memory is a static
// device array of SB2_NOALLOC_SCRATCH_BYTES bytes (each device that runs the
// library holds its own copy until the process ends).  In host code the
// array's name is only a stand-in for its device address: the address is read
// once per device with hipGetSymbolAddress, with that device current, and only
// that pointer is handed to kernels.  The chunk of past times one pass of the
// contraction chain holds is the largest whose workspace fits the array.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[SB2_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
void* g_scratch_ptr[MAX_DEVICES] = {};
std::mutex g_scratch_mu;

// device address of `scratch` on the current device (looked up on first use)
hipError_t scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// largest chunk of past times whose collision workspace fits `cap` bytes (0: none)
int noalloc_chunk(int N, int T, int prec, size_t cap) {
  int hi = coll_plan(N, T, prec).ch.S;
  if (coll_plan(N, T, prec, 1).end > cap) return 0;
  int lo = 1;                                  // fits
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    if (coll_plan(N, T, prec, mid).end <= cap) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
}  // namespace

extern "C" {

int sb2_collision_noalloc(int N, int T, const double* v, const void* h, const void* rho_hist, double dt,
                          void* I_out, void* Sigma_out, int prec, void* stream) {
  if (N < 1 || N > SB2_MAX_N || T < 1 || T > SB2_MAX_T) return SB2_ESHAPE;
  if (!v || !h || !rho_hist || !I_out || !finite_pos(dt)) return SB2_EINVAL;
  SB2_PREC(prec);
  const int S = noalloc_chunk(N, T, prec, SB2_NOALLOC_SCRATCH_BYTES);
  if (S < 1) return SB2_ESCRATCH;
  const CollPlan c = coll_plan(N, T, prec, S);
  SB2_ENTRY();
  void* ws = nullptr;
  SB2_TRY(scratch_ptr(&ws));
  SB2_CHECKS(ws, N, {2, v, (i64)N * N * N * N}, {0, h, 1}, {0, rho_hist, T});
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  cplx* U = reinterpret_cast<cplx*>(at(ws, c.U));
  {
    StageTimer tm(5, s);
    SB2_TRY(propagators(N, T, h, dt, U, reinterpret_cast<cplx*>(at(ws, c.ex1)),
                        reinterpret_cast<cplx*>(at(ws, c.ex2)), s));
  }
  SB2_TRY(collision_core(N, T, v, U, rho_hist, dt, reinterpret_cast<cplx*>(I_out),
                         reinterpret_cast<cplx*>(Sigma_out), prec, c, ws, s));
  return SB2_OK;
}

int sb2_collision_v8(int N, int T, const double* vpacked, const void* h, const void* rho_hist, double dt,
                     void* I_out, void* Sigma_out, int prec, void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || N > SB2_MAX_N || T < 1 || T > SB2_MAX_T) return SB2_ESHAPE;
  if (!vpacked || !h || !rho_hist || !I_out || !ws || !finite_pos(dt)) return SB2_EINVAL;
  SB2_PREC(prec);
  const CollPlan c = coll_plan(N, T, prec);
  if (ws_bytes < c.end) return SB2_EWORKSPACE;
  SB2_ENTRY();
  SB2_CHECKS(ws, N, {2, vpacked, (i64)sb2_v8_count(N)}, {0, h, 1}, {0, rho_hist, T});
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  cplx* U = reinterpret_cast<cplx*>(at(ws, c.U));
  {
    StageTimer tm(5, s);
    SB2_TRY(propagators(N, T, h, dt, U, reinterpret_cast<cplx*>(at(ws, c.ex1)),
                        reinterpret_cast<cplx*>(at(ws, c.ex2)), s));
  }
  SB2_TRY(collision_core(N, T, vpacked, U, rho_hist, dt, reinterpret_cast<cplx*>(I_out),
                         reinterpret_cast<cplx*>(Sigma_out), prec, c, ws, s, true));
  return SB2_OK;
}

int sb2_collision_prop(int N, int T, const double* v, const void* U_hist, const void* rho_hist, double dt,
                       void* I_out, void* Sigma_out, int prec, void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || N > SB2_MAX_N || T < 1 || T > SB2_MAX_T) return SB2_ESHAPE;
  if (!v || !U_hist || !rho_hist || !I_out || !ws || !finite_pos(dt)) return SB2_EINVAL;
  SB2_PREC(prec);
  const CollPlan c = coll_plan(N, T, prec);
  if (ws_bytes < c.end) return SB2_EWORKSPACE;
  SB2_ENTRY();
  SB2_CHECKS(ws, N, {2, v, (i64)N * N * N * N}, {1, U_hist, (i64)T * N * N}, {0, rho_hist, T});
  SB2_TRY(collision_core(N, T, v, reinterpret_cast<const cplx*>(U_hist), rho_hist, dt,
                         reinterpret_cast<cplx*>(I_out), reinterpret_cast<cplx*>(Sigma_out), prec, c, ws,
                         reinterpret_cast<hipStream_t>(stream)));
  return SB2_OK;
}

// Symmetric-basis self-energies of T slices (Eqs. 16-17), in chunks.
hipError_t sigma_symmetric(int N, int T, const double* V, const cplx* G, const cplx* Gb, cplx* S,
                           const VertPlan& p, void* ws, hipStream_t s) {
  const i64 nn = (i64)N * N;
  cplx* Vc = reinterpret_cast<cplx*>(at(ws, p.Vc));
  cplx* P = reinterpret_cast<cplx*>(at(ws, p.P));
  cplx* Q = reinterpret_cast<cplx*>(at(ws, p.Q));
  cplx* R = reinterpret_cast<cplx*>(at(ws, p.R));
  cplx* A = reinterpret_cast<cplx*>(at(ws, p.A));
  cplx* B = reinterpret_cast<cplx*>(at(ws, p.B));
  hipError_t e;
  for (int c0 = 0; c0 < T; c0 += p.chunk) {
    const int c = T - c0 < p.chunk ? T - c0 : p.chunk;
    const cplx* Gc = G + (i64)c0 * nn;
    const cplx* Gbc = Gb + (i64)c0 * nn;
    hipLaunchKernelGGL(k_sym_bubble_in, dim3(blocks((long long)c * nn, 256)), dim3(256), 0, s, N, c, Gc, Gbc, P);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    GemmArgs g = gdef();                                  // Q = V P
    g.M = N; g.N = N; g.K = N;
    g.A = Vc; g.sAm = N; g.sAk = 1; g.sAbh = 0;
    g.B = P; g.sBk = N; g.sBn = 1; g.sBbh = nn;
    g.C = Q; g.sCm = N; g.sCn = 1; g.sCbh = nn;
    if ((e = zgemm(g, c, s)) != hipSuccess) return e;
    g = gdef();                                           // R = V Q^T
    g.M = N; g.N = N; g.K = N;
    g.A = Vc; g.sAm = N; g.sAk = 1; g.sAbh = 0;
    g.B = Q; g.sBk = 1; g.sBn = N; g.sBbh = nn;
    g.C = R; g.sCm = N; g.sCn = 1; g.sCbh = nn;
    if ((e = zgemm(g, c, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sym_exch_in, dim3(blocks((long long)c * nn * N, 256)), dim3(256), 0, s, N, c, V, Gc, Gbc,
                       A);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    g = gdef();                                           // B[k][i] = A[k][i] G[k]: one (N^2 x N) x (N x N)
    g.M = N * N; g.N = N; g.K = N;                        // product per past time, rows (i, l)
    g.A = A; g.sAm = N; g.sAk = 1; g.sAbh = nn * N;
    g.B = Gc; g.sBk = N; g.sBn = 1; g.sBbh = nn;
    g.C = B; g.sCm = N; g.sCn = 1; g.sCbh = nn * N;
    if ((e = zgemm(g, c, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sym_finish, dim3(blocks((long long)c * nn, 256)), dim3(256), 0, s, N, c, V, Gc, R, B,
                       S + (i64)c0 * nn);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // extern "C"

namespace {
// Collision integral of a special vertex from given propagators U[k] =
// U(t, t_k) (Eq. 10 with Eq. 11's propagators supplied), float64: the GKBA
// functions as in collision_core, the self-energies of Eq. 14 or Eqs. 16-17,
// and the sum over past times.
hipError_t collision_vertex_core(int N, int T, int vertex, const double* vparam, const cplx* U, const void* rho_hist,
                                 double dt, cplx* I_out, cplx* Sigma_out, const VertPlan& p, void* ws,
                                 hipStream_t s) {
  const i64 nn = (i64)N * N;
  auto P = [&](size_t off) { return reinterpret_cast<cplx*>(at(ws, off)); };
  hipError_t e;
  {
    StageTimer tm(5, s);
    GemmArgs g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = U; g.sAm = N; g.sAk = 1; g.sAbh = nn;
    g.B = rho_hist; g.sBk = N; g.sBn = 1; g.sBbh = nn;
    g.C = P(p.X); g.sCm = N; g.sCn = 1; g.sCbh = nn;
    if ((e = zgemm(g, T, s)) != hipSuccess) return e;
    g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = rho_hist; g.sAm = N; g.sAk = 1; g.sAbh = nn;
    g.B = U; g.sBk = 1; g.sBn = N; g.sBbh = nn; g.conjB = 1;
    g.C = P(p.Y); g.sCm = N; g.sCn = 1; g.sCbh = nn;
    if ((e = zgemm(g, T, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gkba, dim3(blocks((long long)T * nn, 256)), dim3(256), 0, s, N, T, U, P(p.X), P(p.Y),
                       P(p.Gl), P(p.Gg), P(p.Glb), P(p.Ggb));
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {
    StageTimer tm(6, s);
    if (vertex == SB2_VERTEX_DIAGONAL) {
      const dim3 grid(blocks((long long)T * nn, 256));
      hipLaunchKernelGGL(k_sigma_diag, grid, dim3(256), 0, s, N, T, vparam, P(p.Gl), P(p.Ggb), P(p.Sl));
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_sigma_diag, grid, dim3(256), 0, s, N, T, vparam, P(p.Gg), P(p.Glb), P(p.Sg));
      if ((e = hipGetLastError()) != hipSuccess) return e;
    } else {
      hipLaunchKernelGGL(k_real_to_c, dim3(blocks(nn, 256)), dim3(256), 0, s, nn, vparam, P(p.Vc));
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if ((e = sigma_symmetric(N, T, vparam, P(p.Gl), P(p.Ggb), P(p.Sl), p, ws, s)) != hipSuccess) return e;
      if ((e = sigma_symmetric(N, T, vparam, P(p.Gg), P(p.Glb), P(p.Sg), p, ws, s)) != hipSuccess) return e;
    }
  }
  if (Sigma_out) {
    const size_t bytes = (size_t)T * nn * C128;
    if ((e = hipMemcpyAsync(Sigma_out, P(p.Sl), bytes, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(Sigma_out + (i64)T * nn, P(p.Sg), bytes, hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return e;
  }
  return collision_terms(N, T, P(p.Sl), P(p.Sg), P(p.Glb), P(p.Ggb), P(p.terms), dt, I_out, s);
}

// Time steps n0 .. n_end - 1 of the propagation of Sec. II (Eqs. 8, 11, 12):
// h_HF from hf(rho_n, heff), U_step = exp(-i h_HF dt), I_n from coll(n, U, I)
// over the past times t_0 .. t_{n-1} (I_0 = 0), the exponential-Euler density
// step and the propagator-history update.  hf and coll enqueue their work.
// sqp (optional): a constant correction of the GKBA propagator, whose history
// is then advanced by exp(-i (h_HF + sqp) dt) while the density step keeps
// U_step.
template <class HF, class COLL>
hipError_t propagate_steps(int N, int n0, int n_end, void* rho_hist, void* U_hist, void* I_hist, double dt,
                           int flags, const PropPlan& p, void* ws, hipStream_t s, HF&& hf, COLL&& coll,
                           const cplx* sqp = nullptr) {
  const i64 nn = (i64)N * N;
  const size_t mb = (size_t)nn * C128;
  cplx* rho = reinterpret_cast<cplx*>(rho_hist);
  cplx* U = reinterpret_cast<cplx*>(U_hist);
  cplx* heff = reinterpret_cast<cplx*>(at(ws, p.heff));
  cplx* ustep = reinterpret_cast<cplx*>(at(ws, p.ustep));
  cplx* I = reinterpret_cast<cplx*>(at(ws, p.I));
  cplx* T1 = reinterpret_cast<cplx*>(at(ws, p.T1));
  cplx* ex1 = reinterpret_cast<cplx*>(at(ws, p.ex1));
  cplx* ex2 = reinterpret_cast<cplx*>(at(ws, p.ex2));
  cplx* tmp = reinterpret_cast<cplx*>(at(ws, p.tmp));
  // propagator of the GKBA history: U_step itself, or the corrected step
  cplx* uhist = ustep;
  hipError_t e;
  for (int n = n0; n < n_end; ++n) {
    cplx* rho_n = rho + (i64)n * nn;
    // h_HF(t_n) = h + Sigma_HF(rho_n) (Eq. 12), U_step = exp(-i h_HF dt) (Eq. 11)
    if ((e = hf(rho_n, heff)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_expm, dim3(1), dim3(EXPM_THREADS), 0, s, N, heff, 0.0, -dt, ustep, ex1, ex2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (sqp) {
      cplx* hqp = reinterpret_cast<cplx*>(at(ws, p.hqp));
      uhist = reinterpret_cast<cplx*>(at(ws, p.uqp));
      hipLaunchKernelGGL(k_add_c, dim3(blocks(nn, 256)), dim3(256), 0, s, nn, heff, sqp, hqp);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_expm, dim3(1), dim3(EXPM_THREADS), 0, s, N, hqp, 0.0, -dt, uhist, ex1, ex2);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // I_ns(t_n) over the past times t_0 .. t_{n-1} (Eq. 9)
    if ((flags & SB2_PROP_COLLISION) && n > 0) {
      if ((e = coll(n, U, rho, I)) != hipSuccess) return e;
    } else {
      hipLaunchKernelGGL(k_fill_u32, dim3(blocks(4 * nn, 256)), dim3(256), 0, s, reinterpret_cast<unsigned*>(I),
                         (int)(4 * nn), 0u);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (I_hist && (e = hipMemcpyAsync(reinterpret_cast<cplx*>(I_hist) + (i64)n * nn, I, mb,
                                      hipMemcpyDeviceToDevice, s)) != hipSuccess)
      return e;
    // rho_{n+1} = U_step rho_n U_step^dag - dt (I + I^dag) (Eq. 8, exponential Euler)
    GemmArgs g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = ustep; g.sAm = N; g.sAk = 1;
    g.B = rho_n; g.sBk = N; g.sBn = 1;
    g.C = T1; g.sCm = N; g.sCn = 1;
    if ((e = zgemm(g, 1, s)) != hipSuccess) return e;
    g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = T1; g.sAm = N; g.sAk = 1;
    g.B = ustep; g.sBk = 1; g.sBn = N; g.conjB = 1;
    g.C = ex1; g.sCm = N; g.sCn = 1;
    if ((e = zgemm(g, 1, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_rho_finish, dim3(blocks(nn, 256)), dim3(256), 0, s, N, ex1, I, dt, rho_n + nn);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // U(t_{n+1}, t_k) = U_step U(t_n, t_k) for k < n, U(t_{n+1}, t_n) = U_step
    // (with the corrected step when sqp is given)
    if (n > 0) {
      g = gdef();
      g.M = N; g.N = N; g.K = N;
      g.A = uhist; g.sAm = N; g.sAk = 1; g.sAbh = 0;
      g.B = U; g.sBk = N; g.sBn = 1; g.sBbh = nn;
      g.C = tmp; g.sCm = N; g.sCn = 1; g.sCbh = nn;
      if ((e = zgemm(g, n, s)) != hipSuccess) return e;
      if ((e = hipMemcpyAsync(U, tmp, (size_t)n * mb, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    }
    if ((e = hipMemcpyAsync(U + (i64)n * nn, uhist, mb, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}
}  // namespace

extern "C" {

int sb2_collision_vertex(int N, int T, int vertex, const double* vparam, const void* h, const void* rho_hist,
                         double dt, void* I_out, void* Sigma_out, void* ws, size_t ws_bytes, void* stream) {
  if (N < 1 || N > SB2_MAX_N || T < 1 || T > SB2_MAX_T) return SB2_ESHAPE;
  if (!vparam || !h || !rho_hist || !I_out || !ws || !finite_pos(dt)) return SB2_EINVAL;
  if (vertex != SB2_VERTEX_DIAGONAL && vertex != SB2_VERTEX_SYMMETRIC) return SB2_EINVAL;
  const VertPlan p = vert_plan(N, T, vertex);
  if (ws_bytes < p.end) return SB2_EWORKSPACE;
  SB2_ENTRY();
  SB2_CHECKS(ws, N, {2, vparam, vertex == SB2_VERTEX_DIAGONAL ? (i64)N : (i64)N * N}, {0, h, 1}, {0, rho_hist, T});
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  cplx* U = reinterpret_cast<cplx*>(at(ws, p.U));
  {
    StageTimer tm(5, s);
    SB2_TRY(propagators(N, T, h, dt, U, reinterpret_cast<cplx*>(at(ws, p.ex1)),
                        reinterpret_cast<cplx*>(at(ws, p.ex2)), s));
  }
  SB2_TRY(collision_vertex_core(N, T, vertex, vparam, U, rho_hist, dt, reinterpret_cast<cplx*>(I_out),
                                reinterpret_cast<cplx*>(Sigma_out), p, ws, s));
  return SB2_OK;
}

size_t sb2_v8_count(int N) {
  if (N < 1 || N > SB2_MAX_N) return 0;
  const size_t np = (size_t)N * (N + 1) / 2;
  return np * (np + 1) / 2;
}

int sb2_v8_expand(int N, const double* packed, double* v, void* stream) {
  if (N < 1 || N > SB2_MAX_N) return SB2_ESHAPE;
  if (!packed || !v) return SB2_EINVAL;
  const long long total = (long long)N * N * N * N;
  hipLaunchKernelGGL(k_v8_expand, dim3(blocks(total, 256)), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), N,
                     packed, v);
  SB2_TRY(hipGetLastError());
  return SB2_OK;
}

}  // extern "C"

namespace {
// sb2_gkba_propagate, with an optional coupling history lam[m] = lambda(t_m)
// (the interaction is lambda(t) v: Sigma_HF(t_n) carries lambda(t_n), the
// self-energy Sigma(t_n, t_k) lambda(t_n) lambda(t_k)).
int propagate_general(int N, int n0, int nsteps, const double* v, const void* h, void* rho_hist, void* U_hist,
                      void* I_hist, const double* lam, double dt, int flags, int prec, void* ws, size_t ws_bytes,
                      void* stream, const void* sqp = nullptr) {
  if (N < 1 || N > SB2_MAX_N || n0 < 0 || nsteps < 1 || (long long)n0 + nsteps > SB2_MAX_T) return SB2_ESHAPE;
  if (!v || !h || !rho_hist || !U_hist || !ws || !finite_pos(dt)) return SB2_EINVAL;
  if (flags & ~(SB2_PROP_HF | SB2_PROP_COLLISION)) return SB2_EINVAL;
  SB2_PREC(prec);
  const int n_end = n0 + nsteps;
  const PropPlan p = prop_plan(N, n_end, prec);
  if (ws_bytes < p.end) return SB2_EWORKSPACE;
  SB2_ENTRY();
  SB2_CHECKS(ws, N, {2, v, (i64)N * N * N * N}, {0, h, 1}, {0, rho_hist, n0 + 1}, {1, U_hist, (i64)n0 * N * N},
             {2, lam, lam ? (i64)n_end : 0}, {1, sqp, sqp ? (i64)N * N : 0});
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int now = 0;
  auto hf = [&](const cplx* rho_n, cplx* heff) {
    now = (int)((rho_n - reinterpret_cast<const cplx*>(rho_hist)) / ((i64)N * N));
    hipLaunchKernelGGL(k_sigma_hf, dim3(N), dim3(SIGMA_HF_THREADS), 0, s, N, v, rho_n,
                       reinterpret_cast<const cplx*>(h), (flags & SB2_PROP_HF) ? 1 : 0, heff, lam, now);
    return hipGetLastError();
  };
  auto coll = [&](int n, const cplx* U, const cplx* rho, cplx* I) {
    const CollPlan c = coll_plan(N, n, prec);
    return collision_core(N, n, v, U, rho, dt, I, nullptr, prec, c, ws, s, false, lam, n);
  };
  SB2_TRY(propagate_steps(N, n0, n_end, rho_hist, U_hist, I_hist, dt, flags, p, ws, s, hf, coll,
                          reinterpret_cast<const cplx*>(sqp)));
  return SB2_OK;
}

// sb2_gkba_propagate_linear (see lin_plan for the factorisation).  P (N x N)
// and M (N^4) are the caller's state; at n0 = 0 they start as 1 and 0.
// lam (optional): coupling history; past time k joins M weighted by
// lambda(t_k), I(t_n) and Sigma_HF(t_n) carry lambda(t_n).
int propagate_linear(int N, int n0, int nsteps, const double* v, const void* h, void* rho_hist, void* Pst,
                     void* Mst, void* I_hist, const double* lam, double dt, int flags, void* ws, size_t ws_bytes,
                     void* stream) {
  if (N < 1 || N > SB2_MAX_N || n0 < 0 || nsteps < 1 || (long long)n0 + nsteps > SB2_MAX_T) return SB2_ESHAPE;
  if (!v || !h || !rho_hist || !Pst || !Mst || !ws || !finite_pos(dt)) return SB2_EINVAL;
  if (flags & ~(SB2_PROP_HF | SB2_PROP_COLLISION)) return SB2_EINVAL;
  const LinPlan p = lin_plan(N);
  if (ws_bytes < p.end) return SB2_EWORKSPACE;
  SB2_ENTRY();
  const i64 n = N, n2 = n * n, n3 = n2 * n, n4 = n3 * n;
  SB2_CHECKS(ws, N, {2, v, n4}, {0, h, 1}, {0, rho_hist, n0 + 1}, {1, Pst, n0 > 0 ? n2 : 0},
             {1, Mst, n0 > 0 ? n4 : 0}, {2, lam, lam ? (i64)n0 + nsteps : 0});
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  auto P_ = [&](size_t off) { return reinterpret_cast<cplx*>(at(ws, off)); };
  cplx* rho = reinterpret_cast<cplx*>(rho_hist);
  cplx* P = reinterpret_cast<cplx*>(Pst);
  cplx* M = reinterpret_cast<cplx*>(Mst);
  cplx *heff = P_(p.heff), *ustep = P_(p.ustep), *I = P_(p.I), *T1 = P_(p.T1), *ex1 = P_(p.ex1), *ex2 = P_(p.ex2);
  cplx *padj = P_(p.padj), *X = P_(p.x), *Y = P_(p.y), *Gl = P_(p.gl), *Gg = P_(p.gg), *Glb = P_(p.glb),
       *Ggb = P_(p.ggb), *ptmp = P_(p.ptmp), *ip = P_(p.ip), *r1 = P_(p.r1), *r2 = P_(p.r2), *C3 = P_(p.c3),
       *part = P_(p.part);
  const bool coll = (flags & SB2_PROP_COLLISION) != 0;
  const size_t mb = (size_t)n2 * C128;
  if (n0 == 0) {
    hipLaunchKernelGGL(k_eye_c, dim3(blocks(n2, 256)), dim3(256), 0, s, N, P);
    SB2_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks(4 * n4, 256)), dim3(256), 0, s, reinterpret_cast<unsigned*>(M),
                       (int)(4 * n4), 0u);
    SB2_TRY(hipGetLastError());
  }
  if (coll) SB2_TRY(prep_dispatch(SB2_FP64, N, v, p.ch, ws, s));
  const ChainRefs refs = chain_refs(SB2_FP64, N, 2, p.ch, ws, C3);
  const int n_end = n0 + nsteps;
  for (int t = n0; t < n_end; ++t) {
    cplx* rho_n = rho + (i64)t * n2;
    // h_HF(t_n) and U_step (Eqs. 11, 12)
    hipLaunchKernelGGL(k_sigma_hf, dim3(N), dim3(SIGMA_HF_THREADS), 0, s, N, v, rho_n,
                       reinterpret_cast<const cplx*>(h), (flags & SB2_PROP_HF) ? 1 : 0, heff, lam, t);
    SB2_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_expm, dim3(1), dim3(EXPM_THREADS), 0, s, N, heff, 0.0, -dt, ustep, ex1, ex2);
    SB2_TRY(hipGetLastError());
    if (coll && t > 0) {
      StageTimer tm(7, s);
      // rotated interaction, one leg per product:
      //   r1[n'][i][r][p]  = sum_n P[n][n'] v[i][r][p][n]
      //   r2[r'][n'][i][p] = sum_r conj(P[r][r']) r1[n'][i][r][p]
      //   r1[p'][r'][n'][i] = sum_p P[p][p'] r2[r'][n'][i][p]   = vt_{i r' p' n'}
      GemmArgs g = gdef();
      g.M = N; g.N = (int)n3; g.K = N;
      g.A = P; g.sAm = 1; g.sAk = N;
      g.B = v; g.sBk = 1; g.sBn = N;
      g.C = r1; g.sCm = n3; g.sCn = 1;
      SB2_TRY(zg_m_cr(g, 1, s, N));
      g = gdef();
      g.M = N; g.N = N; g.K = N;
      g.A = P; g.sAm = 1; g.sAk = N; g.conjA = 1;
      g.B = r1; g.sBk = N; g.sBn = 1; g.sBbh = n2;
      g.C = r2; g.sCm = n3; g.sCn = 1; g.sCbh = N;
      SB2_TRY(zg_m(g, (int)n2, s, N));
      g = gdef();
      g.M = N; g.N = (int)n3; g.K = N;
      g.A = P; g.sAm = 1; g.sAk = N;
      g.B = r2; g.sBk = 1; g.sBn = N;
      g.C = r1; g.sCm = n3; g.sCn = 1;
      SB2_TRY(zg_m(g, 1, s, N));
      // ip[i][l] = sum_{(p,r,n)} vt[i][(n,p,r)] M[(p,r,n)][l]   (split-K, float64 sum of the partials)
      g = gdef();
      g.M = N; g.N = N; g.K = (int)n3; g.kchunk = p.kchunk;
      g.A = r1; g.sAm = 1; g.sAk = N;
      g.B = M; g.sBk = N; g.sBn = 1;
      g.C = part; g.sCm = N; g.sCn = 1; g.sCz = n2;
      SB2_TRY(zg_m(g, 1, s, N));
      hipLaunchKernelGGL(k_sum_partials, dim3(blocks(n2, 256)), dim3(256), 0, s, n2, p.nz, part, ip, 0);
      SB2_TRY(hipGetLastError());
      // I = dt ip P^dag
      g = gdef();
      g.M = N; g.N = N; g.K = N;
      g.A = ip; g.sAm = N; g.sAk = 1;
      g.B = P; g.sBk = 1; g.sBn = N; g.conjB = 1;
      g.C = I; g.sCm = N; g.sCn = 1; g.alpha_re = dt;
      SB2_TRY(zgemm(g, 1, s));
      if (lam) {
        hipLaunchKernelGGL(k_scale_by, dim3(blocks(n2, 256)), dim3(256), 0, s, n2, I, lam, t);
        SB2_TRY(hipGetLastError());
      }
    } else {
      hipLaunchKernelGGL(k_fill_u32, dim3(blocks(4 * n2, 256)), dim3(256), 0, s, reinterpret_cast<unsigned*>(I),
                         (int)(4 * n2), 0u);
      SB2_TRY(hipGetLastError());
    }
    if (I_hist) SB2_TRY(hipMemcpyAsync(reinterpret_cast<cplx*>(I_hist) + (i64)t * n2, I, mb,
                                       hipMemcpyDeviceToDevice, s));
    // rho_{n+1} = U_step rho_n U_step^dag - dt (I + I^dag) (Eq. 8)
    GemmArgs g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = ustep; g.sAm = N; g.sAk = 1;
    g.B = rho_n; g.sBk = N; g.sBn = 1;
    g.C = T1; g.sCm = N; g.sCn = 1;
    SB2_TRY(zgemm(g, 1, s));
    g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = T1; g.sAm = N; g.sAk = 1;
    g.B = ustep; g.sBk = 1; g.sBn = N; g.conjB = 1;
    g.C = ex1; g.sCm = N; g.sCn = 1;
    SB2_TRY(zgemm(g, 1, s));
    hipLaunchKernelGGL(k_rho_finish, dim3(blocks(n2, 256)), dim3(256), 0, s, N, ex1, I, dt, rho_n + n2);
    SB2_TRY(hipGetLastError());
    if (coll) {
      StageTimer tm(7, s);
      // past time t joins M: functions a, b, abar, bbar from P_t (the GKBA set-up with U = P_t^dag)
      hipLaunchKernelGGL(k_adjoint_c, dim3(blocks(n2, 256)), dim3(256), 0, s, N, P, padj);
      SB2_TRY(hipGetLastError());
      g = gdef();
      g.M = N; g.N = N; g.K = N;
      g.A = padj; g.sAm = N; g.sAk = 1;
      g.B = rho_n; g.sBk = N; g.sBn = 1;
      g.C = X; g.sCm = N; g.sCn = 1;
      SB2_TRY(zgemm(g, 1, s));
      g.A = rho_n; g.B = P; g.C = Y;
      SB2_TRY(zgemm(g, 1, s));
      hipLaunchKernelGGL(k_gkba, dim3(blocks(n2, 256)), dim3(256), 0, s, N, 1, padj, X, Y, Gl, Gg, Glb, Ggb);
      SB2_TRY(hipGetLastError());
      SB2_TRY(pack_dispatch(SB2_FP64, N, 1, Gl, Gg, Glb, Ggb, 0, p.ch, ws, s));
      SB2_TRY((launch_stage<PK_F64, 0>(refs, s)));
      SB2_TRY((launch_stage<PK_F64, 1>(refs, s)));
      SB2_TRY((launch_stage<PK_F64, 2>(refs, s)));
      // M[(p,r,n)][l] += lambda(t_t) (Ct^>[j][(n,p,r)] abar[j][l] - Ct^<[j][(n,p,r)] bbar[j][l])
      // (the packed chain operands are already taken, so abar and bbar carry the weight)
      if (lam) {
        hipLaunchKernelGGL(k_scale_by, dim3(blocks(n2, 256)), dim3(256), 0, s, n2, Glb, lam, t);
        SB2_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_scale_by, dim3(blocks(n2, 256)), dim3(256), 0, s, n2, Ggb, lam, t);
        SB2_TRY(hipGetLastError());
      }
      for (int sig = 0; sig < 2; ++sig) {
        g = gdef();
        g.M = (int)n3; g.N = N; g.K = N;
        g.A = C3 + (i64)sig * n4; g.sAm = 1; g.sAk = n3;
        g.B = sig ? Glb : Ggb; g.sBk = N; g.sBn = 1;
        g.C = M; g.Mlo = (int)n2; g.sCmh = N; g.sCm = n2; g.sCn = 1;
        g.alpha_re = sig ? 1.0 : -1.0; g.beta1 = 1;
        SB2_TRY(zg_n(g, 1, s, N));
      }
    }
    // P_{n+1} = U_step P_n
    g = gdef();
    g.M = N; g.N = N; g.K = N;
    g.A = ustep; g.sAm = N; g.sAk = 1;
    g.B = P; g.sBk = N; g.sBn = 1;
    g.C = ptmp; g.sCm = N; g.sCn = 1;
    SB2_TRY(zgemm(g, 1, s));
    SB2_TRY(hipMemcpyAsync(P, ptmp, mb, hipMemcpyDeviceToDevice, s));
  }
  return SB2_OK;
}
}  // namespace

extern "C" {

int sb2_gkba_propagate(int N, int n0, int nsteps, const double* v, const void* h, void* rho_hist, void* U_hist,
                       void* I_hist, double dt, int flags, int prec, void* ws, size_t ws_bytes, void* stream) {
  return propagate_general(N, n0, nsteps, v, h, rho_hist, U_hist, I_hist, nullptr, dt, flags, prec, ws, ws_bytes,
                           stream);
}

int sb2_gkba_propagate_switched(int N, int n0, int nsteps, const double* v, const void* h, void* rho_hist,
                                void* U_hist, void* I_hist, const double* lambda, double dt, int flags, int prec,
                                void* ws, size_t ws_bytes, void* stream) {
  if (!lambda) return SB2_EINVAL;
  return propagate_general(N, n0, nsteps, v, h, rho_hist, U_hist, I_hist, lambda, dt, flags, prec, ws, ws_bytes,
                           stream);
}

int sb2_gkba_propagate_linear(int N, int n0, int nsteps, const double* v, const void* h, void* rho_hist, void* P,
                              void* M, void* I_hist, const double* lambda, double dt, int flags, void* ws,
                              size_t ws_bytes, void* stream) {
  return propagate_linear(N, n0, nsteps, v, h, rho_hist, P, M, I_hist, lambda, dt, flags, ws, ws_bytes, stream);
}

int sb2_gkba_propagate_qp(int N, int n0, int nsteps, const double* v, const void* h, const void* sigma_qp,
                          void* rho_hist, void* U_hist, void* I_hist, double dt, int flags, int prec, void* ws,
                          size_t ws_bytes, void* stream) {
  if (!sigma_qp) return SB2_EINVAL;
  return propagate_general(N, n0, nsteps, v, h, rho_hist, U_hist, I_hist, nullptr, dt, flags, prec, ws, ws_bytes,
                           stream, sigma_qp);
}

int sb2_gkba_propagate_vertex(int N, int n0, int nsteps, int vertex, const double* vparam, const void* h,
                              void* rho_hist, void* U_hist, void* I_hist, double dt, int flags, void* ws,
                              size_t ws_bytes, void* stream) {
  if (N < 1 || N > SB2_MAX_N || n0 < 0 || nsteps < 1 || (long long)n0 + nsteps > SB2_MAX_T) return SB2_ESHAPE;
  if (!vparam || !h || !rho_hist || !U_hist || !ws || !finite_pos(dt)) return SB2_EINVAL;
  if (vertex != SB2_VERTEX_DIAGONAL && vertex != SB2_VERTEX_SYMMETRIC) return SB2_EINVAL;
  if (flags & ~(SB2_PROP_HF | SB2_PROP_COLLISION)) return SB2_EINVAL;
  const int n_end = n0 + nsteps;
  const PropPlan p = prop_plan(N, n_end, SB2_FP64, vertex);
  if (ws_bytes < p.end) return SB2_EWORKSPACE;
  SB2_ENTRY();
  SB2_CHECKS(ws, N, {2, vparam, vertex == SB2_VERTEX_DIAGONAL ? (i64)N : (i64)N * N}, {0, h, 1},
             {0, rho_hist, n0 + 1}, {1, U_hist, (i64)n0 * N * N});
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int sym = vertex == SB2_VERTEX_SYMMETRIC ? 1 : 0;
  auto hf = [&](const cplx* rho_n, cplx* heff) {
    hipLaunchKernelGGL(k_sigma_hf_vertex, dim3(blocks((long long)N * N, 256)), dim3(256), 0, s, N, sym, vparam,
                       rho_n, reinterpret_cast<const cplx*>(h), (flags & SB2_PROP_HF) ? 1 : 0, heff);
    return hipGetLastError();
  };
  auto coll = [&](int n, const cplx* U, const cplx* rho, cplx* I) {
    const VertPlan vp = vert_plan(N, n, vertex);
    return collision_vertex_core(N, n, vertex, vparam, U, rho, dt, I, nullptr, vp, ws, s);
  };
  SB2_TRY(propagate_steps(N, n0, n_end, rho_hist, U_hist, I_hist, dt, flags, p, ws, s, hf, coll));
  return SB2_OK;
}

int sb2_rho_step(int N, const void* h, const void* rho, const void* I, double dt, void* rho_out, void* ws,
                 size_t ws_bytes, void* stream) {
  if (N < 1 || N > SB2_MAX_N) return SB2_ESHAPE;
  if (!h || !rho || !I || !rho_out || !ws || !finite_pos(dt)) return SB2_EINVAL;
  if (ws_bytes < rho_plan(N)) return SB2_EWORKSPACE;
  SB2_ENTRY();
  SB2_CHECKS(ws, N, {0, h, 1}, {0, rho, 1}, {1, I, (i64)N * N});
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const size_t m = al((size_t)N * N * C128);
  cplx* U = reinterpret_cast<cplx*>(at(ws, 0));
  cplx* T1 = reinterpret_cast<cplx*>(at(ws, m));
  cplx* ex1 = reinterpret_cast<cplx*>(at(ws, 2 * m));
  cplx* ex2 = reinterpret_cast<cplx*>(at(ws, 3 * m));
  hipLaunchKernelGGL(k_expm, dim3(1), dim3(EXPM_THREADS), 0, s, N, reinterpret_cast<const cplx*>(h), 0.0, -dt, U,
                     ex1, ex2);
  SB2_TRY(hipGetLastError());
  GemmArgs g = gdef();
  g.M = N; g.N = N; g.K = N;
  g.A = U; g.sAm = N; g.sAk = 1;
  g.B = rho; g.sBk = N; g.sBn = 1;
  g.C = T1; g.sCm = N; g.sCn = 1;
  SB2_TRY(zgemm(g, 1, s));
  g = gdef();
  g.M = N; g.N = N; g.K = N;
  g.A = T1; g.sAm = N; g.sAk = 1;
  g.B = U; g.sBk = 1; g.sBn = N; g.conjB = 1;
  g.C = ex1; g.sCm = N; g.sCn = 1;
  SB2_TRY(zgemm(g, 1, s));
  hipLaunchKernelGGL(k_rho_finish, dim3(blocks((long long)N * N, 256)), dim3(256), 0, s, N, ex1,
                     reinterpret_cast<const cplx*>(I), dt, reinterpret_cast<cplx*>(rho_out));
  SB2_TRY(hipGetLastError());
  return SB2_OK;
}

int sb2_collision_backward(int N, int T, const double* v, const void* h, const void* rho_hist, double dt,
                           const void* gI, double* gv, void* gh, void* grho, int prec, void* ws,
                           size_t ws_bytes, void* stream) {
  if (N < 1 || N > SB2_MAX_N || T < 1 || T > SB2_MAX_T) return SB2_ESHAPE;
  if (!v || !h || !rho_hist || !gI || !gv || !gh || !grho || !ws || !finite_pos(dt)) return SB2_EINVAL;
  SB2_PREC(prec);
  if (prec != SB2_FP64) return SB2_EUNSUPPORTED;
  const BwdPlan b = bwd_plan(N, T);
  if (ws_bytes < b.end) return SB2_EWORKSPACE;
  SB2_ENTRY();
  SB2_CHECKS(ws, N, {2, v, (i64)N * N * N * N}, {0, h, 1}, {0, rho_hist, T}, {1, gI, (i64)N * N});
  hipError_t e = collision_backward(N, T, v, h, rho_hist, dt, gI, gv, gh, grho, b, ws,
                                    reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? SB2_OK : SB2_EHIP;
}

int sb2_autotune(int N, int T, const double* v, const void* h, const void* rho_hist, double dt, int prec, void* ws,
                 size_t ws_bytes, void* stream, int* persist_out, int* r4pct_out, int* fused_out) {
  if (N < 1 || N > SB2_MAX_N || T < 1 || T > SB2_MAX_T) return SB2_ESHAPE;
  if (!v || !h || !rho_hist || !ws || !finite_pos(dt)) return SB2_EINVAL;
  SB2_PREC(prec);
  const int Tt = tune_len(N, T, prec);
  const size_t need = tune_bytes(N, T, prec);
  if (ws_bytes < need) return SB2_EWORKSPACE;
  void* Iout = at(ws, need - al((size_t)N * N * C128));     // tail of the workspace: scratch output
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return SB2_EHIP;
  if (hipEventCreate(&b) != hipSuccess) {
    hipEventDestroy(a);
    return SB2_EHIP;
  }
  const TuneCfg saved = tune_of(N, prec);
  // time one evaluation of the tuning workload with configuration tc
  auto trial = [&](const TuneCfg& tc, float& ms) -> int {
    g_tune[{N, prec}] = tc;
    if (hipEventRecord(a, s) != hipSuccess) return SB2_EHIP;
    const int st = sb2_collision(N, Tt, v, h, rho_hist, dt, Iout, nullptr, prec, ws, ws_bytes, stream);
    if (st != SB2_OK) return st;
    if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess) return SB2_EHIP;
    return hipEventElapsedTime(&ms, a, b) == hipSuccess ? SB2_OK : SB2_EHIP;
  };
  TuneCfg best = default_tune(prec);
  float best_ms = 0.f, ms = 0.f;
  int st = trial(best, ms);                       // warm-up
  if (st == SB2_OK) st = trial(best, best_ms);
  // coordinate search: workgroup target first, then the split-K factor
  const int cand_p[] = {256, 512, 768, 1024, 1536, 2048, 3072};
  const int cand_r[] = {50, 150, 200};
  for (int pt : cand_p) {
    if (st != SB2_OK || pt == best.persist) continue;
    TuneCfg tc = best;
    tc.persist = pt;
    st = trial(tc, ms);
    if (st == SB2_OK && ms < best_ms) { best_ms = ms; best = tc; }
  }
  const TuneCfg base = best;
  for (int rp : cand_r) {
    if (st != SB2_OK) continue;
    TuneCfg tc = base;
    tc.r4pct = rp;
    st = trial(tc, ms);
    if (st == SB2_OK && ms < best_ms) { best_ms = ms; best = tc; }
  }
  if (prec == SB2_SPLIT_FP16 && N <= R23_MAX_N) {
    const int cand_f[] = {256, 1024, 2048};
    const TuneCfg base2 = best;
    for (int f : cand_f) {
      if (st != SB2_OK) continue;
      TuneCfg tc = base2;
      tc.r23 = f;
      st = trial(tc, ms);
      if (st == SB2_OK && ms < best_ms) { best_ms = ms; best = tc; }
    }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (st != SB2_OK) {
    g_tune[{N, prec}] = saved;
    return st;
  }
  g_tune[{N, prec}] = best;
  if (persist_out) *persist_out = best.persist;
  if (r4pct_out) *r4pct_out = best.r4pct;
  if (fused_out) *fused_out = best.r23;
  return SB2_OK;
}

int sb2_set_tuning(int N, int prec, int persist, int r4pct, int fused_wgs) {
  if (N < 1 || N > SB2_MAX_N) return SB2_EINVAL;
  SB2_PREC(prec);
  if (persist < 1 || r4pct < 10 || r4pct > 200 || fused_wgs < 0) return SB2_EINVAL;
  TuneCfg tc;
  tc.persist = persist;
  tc.r4pct = r4pct;
  tc.r23 = fused_wgs;
  g_tune[{N, prec}] = tc;
  return SB2_OK;
}

size_t sb2_batched_workspace_size(int nsys, const sb2_system* sys, int prec) {
  if (nsys < 1 || nsys > MAX_GROUP || !sys || !prec_ok(prec)) return 0;
  for (int i = 0; i < nsys; ++i)
    if (sys[i].N < 1 || sys[i].N > SB2_MAX_N || sys[i].T < 1 || sys[i].T > SB2_MAX_T) return 0;
  size_t need = 0;
  for (const auto& bk : size_buckets(nsys, sys)) need = std::max(need, batch_plan((int)bk.size(), bk.data(), prec).end);
  for (int i = 0; i < nsys; ++i)
    if (batch_solo(sys[i])) need = std::max(need, coll_plan(sys[i].N, sys[i].T, prec).end);
  return need;
}

int sb2_collision_batched(int nsys, const sb2_system* sys, int prec, void* ws, size_t ws_bytes, void* stream) {
  if (nsys < 1 || !sys || !ws) return SB2_EINVAL;
  if (nsys > MAX_GROUP) return SB2_ESHAPE;
  for (int b = 0; b < nsys; ++b) {
    const sb2_system& q = sys[b];
    if (q.N < 1 || q.N > SB2_MAX_N || q.T < 1 || q.T > SB2_MAX_T) return SB2_ESHAPE;
    if (!q.v || !q.h || !q.rho_hist || !q.I_out || !finite_pos(q.dt)) return SB2_EINVAL;
  }
  SB2_PREC(prec);
  // systems of one 16-wide bucket of N share the rounds (and the whole
  // intermediate budget); the buckets, then the solo systems, run one after
  // the other in one enqueue
  const auto buckets = size_buckets(nsys, sys);
  std::vector<BatchPlan> plans;
  for (const auto& bk : buckets) {
    plans.push_back(batch_plan((int)bk.size(), bk.data(), prec));
    if (ws_bytes < plans.back().end) return SB2_EWORKSPACE;
  }
  for (int b = 0; b < nsys; ++b)
    if (batch_solo(sys[b]) && ws_bytes < coll_plan(sys[b].N, sys[b].T, prec).end) return SB2_EWORKSPACE;
  SB2_ENTRY();
  for (int b = 0; b < nsys; ++b) {
    const sb2_system& q = sys[b];
    SB2_CHECKS(ws, q.N, {2, q.v, (i64)q.N * q.N * q.N * q.N}, {0, q.h, 1}, {0, q.rho_hist, q.T});
  }
  for (size_t i = 0; i < buckets.size(); ++i) {
    const hipError_t e = collision_batched((int)buckets[i].size(), buckets[i].data(), prec, plans[i], ws,
                                           reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return SB2_EHIP;
  }
  for (int b = 0; b < nsys; ++b) {
    if (!batch_solo(sys[b])) continue;
    const sb2_system& q = sys[b];
    const int st = sb2_collision(q.N, q.T, q.v, q.h, q.rho_hist, q.dt, q.I_out, nullptr, prec, ws, ws_bytes, stream);
    if (st != SB2_OK) return st;
  }
  return SB2_OK;
}

}  // extern "C"
