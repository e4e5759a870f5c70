// The four stages of the second-Born contraction chain as a single table of
// (operand layout, kernel configuration) entries, used by the direct
// per-system launches and by the grouped multi-system launches alike.
//
//   R1  A[(b,n)][(j,s,q)] = sum_m G[(b,n)][m] W_T[(j,s,q)][m]
//   R2  B[b][n][p][(j,s)] = sum_q G_b[p][q] A[b][n][(j,s)][q]
//   R3  C[b][j][n][p][r]  = sum_s B[b][(n,p,j)][s] GbT_b[r][s]
//   R4  part[z][i][(b,j)] = sum_{k in chunk z} Vp[i][k] C[(b,j)][k],  k = (n,p,r)
#pragma once
#include "stream_gemm.hpp"

namespace sb2 {

enum ScaleWord { S_GMAX = 0, S_GBMAX, S_WMAX, S_VMAX, S_AMAX, S_BMAX, S_CMAX, S_NWORDS };
// After the scale words: a 1 KiB sink (16 bytes per lane of a wave) that
// takes the stores of out-of-range tile elements, so that a tile's stores are
// issued unconditionally (a fixed number per wave).
constexpr int S_TRASH = 64, S_TRASH_WORDS = 256;

// Everything a chain stage needs to know about one system's current chunk.
struct ChainRefs {
  int N, ns;                 // basis size, slices in this chunk (2 per past time)
  int prec;                  // 0 float64, 1 float32, 2 split float16
  int kchunk;                // R4 split-K chunk
  i64 KpW, KpV;              // row pitches of W_T and Vp
  const void* Gs;
  const void* GbT;
  const void* W;
  const void* Vp;
  void* X1;                  // A, then (unless C3 given) C
  void* X2;                  // B
  void* C3;                  // optional separate C buffer (adjoint keeps A, B and C)
  void* part;                // R4 split-K partials
  unsigned* scal;            // split-float16 scale words
  int chunked;               // n-chunked Vp / C layout (fused split-float16 path)
  i64 KB;                    // n-block pitch of the chunked Vp rows
};

__host__ __device__ inline StreamArgs sargs_zero() {
  StreamArgs g;
  char* p = reinterpret_cast<char*>(&g);
  for (unsigned i = 0; i < sizeof(g); ++i) p[i] = 0;
  g.nbl = 1;
  g.kpromote = 4;
  return g;
}

// Operand layout of `stage` (0..3) for the chunk described by r; nbatch gets
// the batch count of the launch.
__host__ __device__ inline StreamArgs stage_args(int stage, const ChainRefs& r, int& nbatch) {
  const i64 n = r.N, n2 = n * n, n3 = n2 * n, n4 = n3 * n;
  const bool h16 = r.prec == 2;
  StreamArgs g = sargs_zero();
  g.trash = r.scal + S_TRASH;
  void* Cc = r.C3 ? r.C3 : r.X1;
  nbatch = 1;
  if (stage == 0) {
    g.M = r.ns * r.N; g.N = (int)n3; g.K = r.N;
    g.S = r.Gs; g.sSs = n;
    g.X = r.W; g.sXx = r.KpW; g.sXplane = n3 * r.KpW;
    g.C = r.X1; g.sCm = n3; g.sCn = 1;
    if (h16) { g.smax = r.scal + S_GMAX; g.xmax = r.scal + S_WMAX; g.cmax = r.scal + S_AMAX; }
  } else if (stage == 1) {
    g.M = r.N; g.N = (int)n2; g.K = r.N; g.nbl = r.N;
    g.S = r.Gs; g.sSs = n; g.sSbh = n2; g.sSbl = 0;
    g.X = r.X1; g.sXx = n; g.sXbh = n4; g.sXbl = n3;
    g.C = r.X2; g.sCm = n2; g.sCn = 1; g.sCbh = n4; g.sCbl = n3;
    if (h16) { g.smax = r.scal + S_GMAX; g.xmax = r.scal + S_AMAX; g.cmax = r.scal + S_BMAX; }
    nbatch = r.ns * r.N;
  } else if (stage == 2) {
    g.M = (int)n3; g.N = r.N; g.K = r.N;
    g.X = r.X2; g.sXx = n; g.sXbh = n4;
    g.S = r.GbT; g.sSs = n; g.sSbh = n2;
    g.C = Cc; g.Mlo = r.N; g.sCmh = n; g.sCm = n3; g.sCn = 1; g.sCbh = n4;
    if (h16) { g.xmax = r.scal + S_BMAX; g.smax = r.scal + S_GBMAX; g.cmax = r.scal + S_CMAX; }
    nbatch = r.ns;
  } else {
    g.M = r.N; g.N = r.ns * r.N; g.K = (int)n3; g.kchunk = r.kchunk;
    g.S = r.Vp; g.sSs = r.KpV; g.sSplane = n * r.KpV;
    g.X = Cc; g.sXx = n3;
    g.C = r.part; g.sCm = (i64)r.ns * r.N; g.sCn = 1; g.sCz = n * r.ns * r.N;
    if (h16) { g.smax = r.scal + S_VMAX; g.xmax = r.scal + S_CMAX; g.kpromote = 2; }
  }
  if (g.kchunk <= 0) g.kchunk = g.K > 0 ? g.K : 1;
  return g;
}

// Kernel configuration of (precision, stage).  ONE: single-slab kernel with
// 8 waves (k_stream1); otherwise the slab-walking kernel (k_stream).
template <int PK, int STAGE> struct StageCfg;
// float64: slab-walking kernel throughout
template <> struct StageCfg<PK_F64, 0> { static constexpr bool ONE = false, SA = true, SC = true, XC = false, ACC64 = false; static constexpr int FS = 4, FX = 2, NW = 4, KS = 112; using Out = double; };
template <> struct StageCfg<PK_F64, 1> { static constexpr bool ONE = false, SA = true, SC = true, XC = true, ACC64 = false; static constexpr int FS = 7, FX = 1, NW = 4, KS = 64; using Out = double; };
template <> struct StageCfg<PK_F64, 2> { static constexpr bool ONE = false, SA = false, SC = true, XC = true, ACC64 = false; static constexpr int FS = 7, FX = 1, NW = 4, KS = 64; using Out = double; };
template <> struct StageCfg<PK_F64, 3> { static constexpr bool ONE = false, SA = true, SC = false, XC = true, ACC64 = false; static constexpr int FS = 7, FX = 1, NW = 4, KS = 32; using Out = double; };
// float32
template <> struct StageCfg<PK_F32, 0> { static constexpr bool ONE = true, SA = true, SC = true, XC = false, ACC64 = false; static constexpr int FS = 8, FX = 1, NW = 8, KS = 128; using Out = float; };
template <> struct StageCfg<PK_F32, 1> { static constexpr bool ONE = true, SA = true, SC = true, XC = true, ACC64 = false; static constexpr int FS = 7, FX = 1, NW = 8, KS = 128; using Out = float; };
template <> struct StageCfg<PK_F32, 2> { static constexpr bool ONE = true, SA = false, SC = true, XC = true, ACC64 = false; static constexpr int FS = 7, FX = 1, NW = 8, KS = 128; using Out = float; };
template <> struct StageCfg<PK_F32, 3> { static constexpr bool ONE = false, SA = true, SC = false, XC = true, ACC64 = true; static constexpr int FS = 7, FX = 1, NW = 4, KS = 64; using Out = double; };
// split float16
template <> struct StageCfg<PK_H16, 0> { static constexpr bool ONE = true, SA = true, SC = true, XC = false, ACC64 = false; static constexpr int FS = 8, FX = 1, NW = 8, KS = 128; using Out = float; };
template <> struct StageCfg<PK_H16, 1> { static constexpr bool ONE = true, SA = true, SC = true, XC = true, ACC64 = false; static constexpr int FS = 7, FX = 1, NW = 8, KS = 128; using Out = float; };
template <> struct StageCfg<PK_H16, 2> { static constexpr bool ONE = true, SA = false, SC = true, XC = true, ACC64 = false; static constexpr int FS = 7, FX = 1, NW = 8, KS = 128; using Out = float; };
template <> struct StageCfg<PK_H16, 3> { static constexpr bool ONE = false, SA = true, SC = false, XC = true, ACC64 = true; static constexpr int FS = 7, FX = 1, NW = 4, KS = 128; using Out = double; };

// The configuration with the shared tile's height set to FSN 16-row fragments
// (FSN = 0: the table's default).  Stages 1-3 share an operand with N rows
// (G_b, Gbar_b, V'), so their tile follows the basis size (16 ceil(N/16)
// rows instead of always 112): at N = 64 a 112-row tile would spend 3/7 of its
// products on padding.  Stage 0 shares the 2 S N rows of the stacked G.
template <int PK, int STAGE, int FSN>
struct StageCfgN : StageCfg<PK, STAGE> {
  static constexpr int FS = (STAGE == 0 || FSN == 0) ? StageCfg<PK, STAGE>::FS : FSN;
};

// Tile height (16-row fragments) of stages 1-3 for basis size N: the smallest
// of 2, 4, 6, 7, 8 that covers N (the instantiated variants).
__host__ __device__ inline int stage_fs(int N) {
  return N <= 32 ? 2 : N <= 64 ? 4 : N <= 96 ? 6 : N <= 112 ? 7 : 8;
}

// Launch geometry of one stage: grid = (tiles_s * npersist, nbatch, nz).
struct StageGeom {
  int tiles_s, tiles_x, npersist, nbatch, nz;
  __host__ __device__ long long blocks() const { return (long long)tiles_s * npersist * nbatch * nz; }
};

template <int PK, int STAGE, int FSN = 0>
__host__ __device__ inline StageGeom stage_geom(StreamArgs& g, int nbatch, int persist_target) {
  using C = StageCfgN<PK, STAGE, FSN>;
  constexpr int SR = 16 * C::FS;
  constexpr int XT = 16 * C::FX * C::NW;
  const int slim = C::SA ? g.M : g.N, xlim = C::SA ? g.N : g.M;
  StageGeom q;
  q.tiles_s = (slim + SR - 1) / SR;
  q.tiles_x = (xlim + XT - 1) / XT;
  q.nbatch = nbatch;
  q.nz = g.K > 0 ? (g.K + g.kchunk - 1) / g.kchunk : 1;
  q.npersist = q.tiles_x;
  if (g.kchunk <= C::KS) {
    const long long want = (persist_target + (long long)q.tiles_s * nbatch - 1) / ((long long)q.tiles_s * nbatch);
    q.npersist = (int)(want < 1 ? 1 : (want > q.tiles_x ? q.tiles_x : want));
  }
  if (C::ONE) q.nz = 1;
  g.tiles_m = q.tiles_s;
  return q;
}

template <int PK, int STAGE, int FSN = 0>
__device__ __forceinline__ void run_stage_block(const StreamArgs& g, const StageGeom& q, long long local) {
  using C = StageCfgN<PK, STAGE, FSN>;
  const long long gx = (long long)q.tiles_s * q.npersist;
  const int bx = (int)(local % gx);
  const long long rest = local / gx;
  const int by = (int)(rest % q.nbatch);
  const int bz = (int)(rest / q.nbatch);
  if constexpr (C::ONE)
    stream1_body<PK, C::SA, C::SC, C::XC, C::FS, C::NW, C::KS, typename C::Out>(g, bx, by, q.npersist);
  else
    stream_body<PK, C::SA, C::SC, C::XC, C::FS, C::FX, C::NW, C::KS, C::ACC64, typename C::Out>(g, bx, by, bz,
                                                                                                 q.npersist);
}

template <int PK, int STAGE, int FSN = 0>
__global__ void __launch_bounds__((64 * StageCfg<PK, STAGE>::NW)) k_stage(const StreamArgs g, const StageGeom q) {
  const long long gx = (long long)q.tiles_s * q.npersist;
  run_stage_block<PK, STAGE, FSN>(g, q,
                                  (long long)blockIdx.x + gx * ((long long)blockIdx.y + (long long)q.nbatch * blockIdx.z));
}

// ---------------------------------------------------------------------------
// Grouped launches over several systems: member i owns blocks
// [off[i], off[i+1]) of a one-dimensional grid and the chunk refs[i] (read
// from device memory); each workgroup finds its member by a scan of off.
// ---------------------------------------------------------------------------
constexpr int MAX_GROUP = 64;

struct GroupTable {
  int count;
  int persist[MAX_GROUP];     // per-member workgroup target of single-slab stages
  long long off[MAX_GROUP + 1];
};

// All members of one grouped launch share the tile height FSN (the batched
// path groups systems by ceil(N/16)).
template <int PK, int STAGE, int FSN = 0>
__global__ void __launch_bounds__((64 * StageCfg<PK, STAGE>::NW))
k_stage_group(const ChainRefs* __restrict__ refs, const GroupTable t) {
  const long long b = blockIdx.x;
  int i = 0;
  while (i + 1 < t.count && b >= t.off[i + 1]) ++i;
  const ChainRefs r = refs[i];
  int nbatch;
  StreamArgs g = stage_args(STAGE, r, nbatch);
  const StageGeom q = stage_geom<PK, STAGE, FSN>(g, nbatch, t.persist[i]);
  run_stage_block<PK, STAGE, FSN>(g, q, b - t.off[i]);
}

// Write a table of chain refs into device memory (the table travels as kernel
// arguments, so the sequence stays valid under stream capture).
constexpr int REFS_PER_WRITE = 24;
struct RefsChunk {
  int count;
  ChainRefs r[REFS_PER_WRITE];
};
__global__ void k_write_refs(ChainRefs* __restrict__ dst, const RefsChunk c) {
  const int i = threadIdx.x;
  if (i < c.count) dst[i] = c.r[i];
}

}  // namespace sb2
