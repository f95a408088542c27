// FP64 direct solve of the reduced interface system (eq. (hps_reduced)) in
// nested-dissection order, the first of the two solvers of Sec. 2.
//
// Planning (host): the nx x ny leaf grid is bisected recursively, the longer
// side first.  A box's exterior list E holds the unknown edge nodes on its
// boundary (nodes on the outer boundary carry Dirichlet data and are never
// unknowns).  Bisecting box b into halves a and c, the separator s is the
// set of nodes both halves have on their boundary (the leaf edges along the
// cut), and E_b = (E_a \ s) ++ (E_c \ s).  A leaf's exterior lists its
// unknown edge nodes, and its Schur complement is its own S restricted to
// them.
//
// Leaves may differ in order (Sec. 2: p from a fixed set).  A shared edge
// then carries the nodes of its lower-order leaf; the other leaf sees the
// polynomial through them at its own nodes (P) and returns its flux through
// the polynomial through its own values (R), so its Schur complement in the
// edge basis is R S P (k_nd_leaf_transform) and its right-hand side R r.
// With one order everywhere no leaf is transformed.
//
// Factorisation (device), level by level from the leaves up; the fronts of
// one level are independent and run as one batch:
//   F     = T_a (+) T_c on [s | E_b]  (each half's Schur complement, scattered)
//   F_ss  = P L U                     (partial pivoting within the front)
//   X     = F_ss^{-1} F_se
//   T_b   = F_ee - F_es X             (passed to the parent)
// Solve: leaf right-hand sides r_t = -(w_t + S_t[:, D] g_D) on the unknown
// slots, the same scatter and elimination upwards (y_b = F_ss^{-1} r_s,
// r_b = r_e - F_es y_b), then from the root down u_s = y_b - X u_E.
//
// Layouts: every front matrix is row-major and dense; the whole tree lives
// in one FP64 arena and one int arena (maps, node ids, pivot order).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <map>
#include <new>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/hps_iface.h"
#include "hps_internal.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kMaxSep = HPS_IFACE_MAX_SEPARATOR;
constexpr int kFactorThreads = 512;   // LU of one separator block per workgroup
constexpr int kSolveThreads = 512;    // 16 right-hand sides per workgroup
constexpr int kSplitLU = 256;         // separators from this size: LU in two launches per panel

// One front as the kernels see it.  Offsets are in doubles or ints.  A
// child's Schur complement and reduced right-hand side live in the FP64
// arena (kind 0: a front, or a transformed leaf) or in the caller's S and
// the leaf right-hand sides (kind 1: a leaf taken as it is).
struct Front {
  long long fss, x, fes, t, y, r;
  long long ca, cc;   // children's Schur complements
  long long ra, rc;   // children's reduced right-hand sides
  int ka, kc;         // kinds of the two children
  int lda, ldc;       // leading dimensions of the children's Schur complements
  int map;            // int arena: map_a [nS+nE], then map_c [nS+nE]
  int gid;            // int arena: global node ids, separator then exterior
  int perm;           // int arena: pivot order of the LU of F_ss [nS]
  int nS, nE;
};

// One side of a leaf: the first global node of its edge and the edge's node
// count; P [m][me] and R [me][m] are offsets into the interpolation table,
// -1 where the edge carries the leaf's own nodes.
struct Side {
  int node0, me, P, R, dir;
};

struct LeafD {
  long long s_off, b_off;   // the leaf's S and boundary slots in the caller's arrays
  long long t_off, r_off;   // transformed leaves: R S P [ne][ne] and R r [ne] in the arena
  int m, ne;                // nodes per side; unknowns of its interface sides (edge basis)
  Side side[4];             // W, E, S, N
};

__device__ __forceinline__ d4 mma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ const double *child_T(const Front &f, bool first, const double *ar,
                                                 const double *S) {
  return ((first ? f.ka : f.kc) ? S : ar) + (first ? f.ca : f.cc);
}

__device__ __forceinline__ const double *child_r(const Front &f, bool first, const double *ar,
                                                 const double *rl) {
  return ((first ? f.ka : f.kc) ? rl : ar) + (first ? f.ra : f.rc);
}

// Side and index of column c of a transformed leaf's edge basis (its
// interface sides in the order W, E, S, N).
__device__ __forceinline__ void edge_basis(const LeafD &L, int c, int &s, int &i) {
  s = 0;
  for (; s < 4; ++s) {
    if (L.side[s].dir) continue;
    if (c < L.side[s].me) break;
    c -= L.side[s].me;
  }
  i = c;
}

// ---------------------------------------------------------------------------
// assembly of the fronts of one level: F = T_a (+) T_c
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_nd_front(const Front *fr, int first, double *ar,
                                                  const int *ia, const double *S) {
  const Front f = fr[first + blockIdx.y];
  const int nS = f.nS, nE = f.nE, n = nS + nE;
  const long long tot = (long long)n * n;
  const double *Ta = child_T(f, true, ar, S);
  const double *Tc = child_T(f, false, ar, S);
  const int *ma = ia + f.map, *mc = ma + n;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < tot;
       e += (long long)gridDim.x * 256) {
    const int i = (int)(e / n), j = (int)(e - (long long)i * n);
    const int ai = ma[i], aj = ma[j], ci = mc[i], cj = mc[j];
    double v = 0.0;
    if (ai >= 0 && aj >= 0) v = Ta[(size_t)ai * f.lda + aj];
    if (ci >= 0 && cj >= 0) v += Tc[(size_t)ci * f.ldc + cj];
    if (i < nS) {
      if (j < nS) ar[f.fss + (size_t)i * nS + j] = v;
      else ar[f.x + (size_t)i * nE + (j - nS)] = v;
    } else {
      if (j < nS) ar[f.fes + (size_t)(i - nS) * nS + j] = v;
      else ar[f.t + (size_t)(i - nS) * nE + (j - nS)] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// leaves on an order boundary: their Schur complement in the edge basis,
// T = R S P over their interface sides (U = S P staged in LDS)
// ---------------------------------------------------------------------------
size_t transform_lds(int m, int ne) { return sizeof(double) * (size_t)(4 * m) * ne; }

__global__ __launch_bounds__(256) void k_nd_leaf_transform(const LeafD *ld, const int *tlist,
                                                           const double *S, const double *tab,
                                                           double *ar) {
  extern __shared__ double U[];   // [nb][ne]
  const LeafD &L = ld[tlist[blockIdx.x]];
  const int m = L.m, nb = 4 * m, ne = L.ne;
  const double *Sl = S + L.s_off;
  for (int e = threadIdx.x; e < nb * ne; e += 256) {
    const int r = e / ne, c = e - r * ne;
    int q, j;
    edge_basis(L, c, q, j);
    const Side sd = L.side[q];
    const double *row = Sl + (size_t)r * nb + q * m;
    double v = 0.0;
    if (sd.P < 0) {
      v = row[j];
    } else {
      for (int l = 0; l < m; ++l) v += row[l] * tab[sd.P + l * sd.me + j];
    }
    U[e] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < ne * ne; e += 256) {
    const int a = e / ne, c = e - a * ne;
    int s, i;
    edge_basis(L, a, s, i);
    const Side sd = L.side[s];
    double v = 0.0;
    if (sd.R < 0) {
      v = U[(s * m + i) * ne + c];
    } else {
      for (int k = 0; k < m; ++k) v += tab[sd.R + i * m + k] * U[(s * m + k) * ne + c];
    }
    ar[L.t_off + e] = v;
  }
}

// ---------------------------------------------------------------------------
// LU with partial pivoting of F_ss, one front per workgroup.  Right-looking
// over 16-column panels: the panel is factored in LDS (largest magnitude in
// the column, ties to the lowest row, as LAPACK getrf), its row exchanges
// are applied to the other columns, U12 = L11^{-1} A12, and the trailing
// block is updated with FP64 MFMA in strips of 16 x 64.  The final row order
// is written to `perm` (row i of P F_ss is row perm[i] of F_ss).
// ---------------------------------------------------------------------------
// Workspace of the register-resident panel elimination behind the callers'
// own LDS: the wavefronts' candidate keys and rows (two slots by column
// parity), the pivots as panel rows, and the row order while the panel's
// exchanges are formed.
struct PanelSlots {
  unsigned long long *key;   // [2][NW] candidate keys (0: none)
  double *vals;              // [2][NW][16] candidate rows' values
  int *pivo;                 // [16] pivot of each column as a panel row (before exchanges)
  int *at, *where;           // [rows] panel row at each place, place of each panel row
};

size_t panel_slot_bytes(int n) {
  const int nw = kFactorThreads / 64;
  return 16 + sizeof(unsigned long long) * 2 * nw + sizeof(double) * 2 * nw * 16 +
         sizeof(int) * (16 + 2 * (size_t)n);
}

__device__ __forceinline__ PanelSlots panel_slots(void *end_of_callers) {
  constexpr int NW = kFactorThreads / 64;
  const size_t a = ((size_t)end_of_callers + 15) & ~(size_t)15;
  PanelSlots ps;
  ps.key = (unsigned long long *)a;
  ps.vals = (double *)(ps.key + 2 * NW);
  ps.pivo = (int *)(ps.vals + 2 * NW * 16);
  ps.at = ps.pivo + 16;
  ps.where = nullptr;   // set by the caller from the row count
  return ps;
}

size_t getrf_lds(int n) {
  const int n16 = (n + 15) & ~15;
  const int nw = kFactorThreads / 64;
  return sizeof(double) * ((size_t)n16 * 16 + nw) + sizeof(int) * (nw + 16 + (size_t)n + 1) +
         panel_slot_bytes(n);
}

// Pivot search key of a panel row: the magnitude's leading bits (the top 32
// of the FP64 pattern: exponent and 20 mantissa bits; NaN above infinity),
// then the complemented row, so that the maximum is unique and near-ties
// go to the lowest row.  0 marks "no candidate".
__device__ __forceinline__ unsigned long long nd_key(double v, int r) {
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(fabs(v)) >> 32);
  return ((unsigned long long)hi << 32) | (unsigned)(0x7fffffff - r);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long nd_dpp_max(unsigned long long v) {
  const int lo = (int)(unsigned)v, hi = (int)(unsigned)(v >> 32);
  const int olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xf, false);
  const int ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xf, false);
  const unsigned long long o = ((unsigned long long)(unsigned)ohi << 32) | (unsigned)olo;
  return o > v ? o : v;
}

// Wavefront maximum (quad permutations, row shifts, the row broadcasts of
// lanes 15 and 31; lane 63 ends with it), read back to every lane.
__device__ __forceinline__ unsigned long long nd_wave_max(unsigned long long v) {
  v = nd_dpp_max<0xb1, 0xf>(v);
  v = nd_dpp_max<0x4e, 0xf>(v);
  v = nd_dpp_max<0x114, 0xf>(v);
  v = nd_dpp_max<0x118, 0xf>(v);
  v = nd_dpp_max<0x142, 0xa>(v);
  v = nd_dpp_max<0x143, 0xc>(v);
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)v, 63);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

// Each wavefront's candidate for panel column C (over its active rows) and
// that row's values, written by the lane that holds it.
template <int NT, int RPT, int C>
__device__ __forceinline__ void nd_publish(const double (&v)[RPT][16], const bool (&act)[RPT],
                                           int tid, const PanelSlots &ps) {
  constexpr int NW = NT / 64;
  const int lane = tid & 63, wv = tid >> 6, slot = (C & 1) * NW + wv;
  unsigned long long key = 0;
#pragma unroll
  for (int h = 0; h < RPT; ++h) {
    if (act[h]) {
      const unsigned long long kh = nd_key(v[h][C], tid + h * NT);
      key = kh > key ? kh : key;
    }
  }
  const unsigned long long wk = nd_wave_max(key);
  const int wr = 0x7fffffff - (int)(unsigned)(wk & 0xffffffffu);   // INT_MAX: none
  double *dst = ps.vals + slot * 16;
  if (lane == 0) ps.key[slot] = wk;
  if (wk == 0 && lane < 16) dst[lane] = 0.0;
#pragma unroll
  for (int h = 0; h < RPT; ++h) {
    if (tid + h * NT == wr) {
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) dst[cc] = v[h][cc];
    }
  }
}

// Column C of the panel: the pivot is the largest of the wavefronts' keys;
// every thread eliminates its active rows in registers and publishes the
// next column's candidates before the one barrier.
template <int NT, int RPT, int C>
__device__ __forceinline__ void nd_column(double (&v)[RPT][16], bool (&act)[RPT], int tid,
                                          int rows, int w, int c0, const PanelSlots &ps, int *zp) {
  if (C >= w) return;
  constexpr int NW = NT / 64;
  const int s0 = (C & 1) * NW;
  unsigned long long best = ps.key[s0];
  double pval = ps.vals[s0 * 16 + C];
  int bw = 0;
#pragma unroll
  for (int k = 1; k < NW; ++k) {
    const unsigned long long ok = ps.key[s0 + k];
    const double ov = ps.vals[(s0 + k) * 16 + C];
    if (ok > best) {
      best = ok;
      pval = ov;
      bw = k;
    }
  }
  // at least one row is active, so the key names a valid row; the clamp
  // only guards the memory accesses
  const int bi = 0x7fffffff - (int)(unsigned)(best & 0xffffffffu);
  const int pr = (bi >= 0 && bi < rows) ? bi : 0;
  const double *prow = ps.vals + (s0 + bw) * 16;
  if (tid == 0) {
    ps.pivo[C] = pr;
    if (!(fabs(pval) > 0.0) && *zp == 0) *zp = c0 + C + 1;
  }
  const bool doit = pval != 0.0;
  const double inv = doit ? 1.0 / pval : 0.0;
  bool upd[RPT];
  double l[RPT];
#pragma unroll
  for (int h = 0; h < RPT; ++h) {
    const bool mine = tid + h * NT == pr;
    upd[h] = doit && act[h] && !mine;
    if (mine) act[h] = false;
    l[h] = v[h][C] * inv;
    if (upd[h]) v[h][C] = l[h];
  }
#pragma unroll
  for (int cc = C + 1; cc < 16; ++cc) {
    const double u = prow[cc];
#pragma unroll
    for (int h = 0; h < RPT; ++h)
      if (upd[h]) v[h][cc] -= l[h] * u;
  }
  if constexpr (C + 1 < 16) nd_publish<NT, RPT, C + 1>(v, act, tid, ps);
  __syncthreads();
}

template <int NT, int RPT, int... Cs>
__device__ __forceinline__ void nd_columns(double (&v)[RPT][16], bool (&act)[RPT], int tid,
                                           int rows, int w, int c0, const PanelSlots &ps, int *zp,
                                           std::integer_sequence<int, Cs...>) {
  (nd_column<NT, RPT, Cs>(v, act, tid, rows, w, c0, ps, zp), ...);
}

// One 16-column panel of the LU of an n x n row-major A, columns c0 ..
// c0+15, partial pivoting (largest magnitude by the leading 20 mantissa
// bits, ties to the lowest panel row): the panel is eliminated with its
// rows in registers (thread t holds panel rows t and t + NT, one barrier per
// column), the pivots are then turned into the LAPACK sequence of row
// exchanges (pivl; `perm` is the row order: row i of P A is row perm[i] of
// A) and the rows placed accordingly in LDS (P, [n16][16]), the panel
// written back, its exchanges applied to every other column, then U12 =
// L11^{-1} A12.  A zero (or NaN) pivot sets *zp to its column (1-based)
// unless already set.  All threads of the workgroup call it; it ends with a
// barrier.
template <int NT>
__device__ void nd_panel(double *A, int n, int c0, double *P, const PanelSlots &ps0, int *pivl,
                         int *perm, int *zp) {
  constexpr int RPT = (kMaxSep + NT - 1) / NT;
  const int tid = threadIdx.x;
  const int w = min(16, n - c0), rows = n - c0;
  PanelSlots ps = ps0;
  ps.where = ps.at + rows;
  double v[RPT][16];
  bool act[RPT];
#pragma unroll
  for (int h = 0; h < RPT; ++h) {
    const int r = tid + h * NT;
    act[h] = r < rows;
#pragma unroll
    for (int c = 0; c < 16; ++c) v[h][c] = (r < rows && c < w) ? A[(size_t)(c0 + r) * n + c0 + c] : 0.0;
  }
  nd_publish<NT, RPT, 0>(v, act, tid, ps);
  __syncthreads();
  nd_columns<NT, RPT>(v, act, tid, rows, w, c0, ps, zp, std::make_integer_sequence<int, 16>());
  // the exchanges in LAPACK's order: at column lc the pivot's current place
  // swaps with place lc
  for (int i = tid; i < rows; i += NT) {
    ps.at[i] = i;
    ps.where[i] = i;
  }
  __syncthreads();
  if (tid == 0) {
    for (int lc = 0; lc < w; ++lc) {
      const int pr = ps.pivo[lc], cur = ps.where[pr], a = ps.at[lc];
      ps.at[lc] = pr;
      ps.where[pr] = lc;
      ps.at[cur] = a;
      ps.where[a] = cur;
      pivl[lc] = c0 + cur;
      if (cur != lc) {
        const int t = perm[c0 + lc];
        perm[c0 + lc] = perm[c0 + cur];
        perm[c0 + cur] = t;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < RPT; ++h) {
    const int r = tid + h * NT;
    if (r < rows) {
      const int d = ps.where[r];
#pragma unroll
      for (int c = 0; c < 16; ++c) P[d * 16 + c] = v[h][c];
    }
  }
  __syncthreads();
  // panel back, and its row exchanges applied to every other column
  for (int e = tid; e < rows * 16; e += NT) {
    const int r = e >> 4, c = e & 15;
    if (c < w) A[(size_t)(c0 + r) * n + c0 + c] = P[e];
  }
  for (int j = tid; j < n; j += NT) {
    if (j >= c0 && j < c0 + w) continue;
    for (int lc = 0; lc < w; ++lc) {
      const int r2 = pivl[lc];
      if (r2 != c0 + lc) {
        double *a = A + (size_t)(c0 + lc) * n + j;
        double *b = A + (size_t)r2 * n + j;
        const double t = *a;
        *a = *b;
        *b = t;
      }
    }
  }
  __syncthreads();
  if (c0 + 16 >= n) return;   // last panel: nothing to the right
  // U12 = L11^{-1} A12 (unit lower L11 from the panel)
  for (int j = c0 + 16 + tid; j < n; j += NT) {
    double x[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) x[k] = A[(size_t)(c0 + k) * n + j];
#pragma unroll
    for (int k = 1; k < 16; ++k) {
      // one row of L11 at a time (keeps its loads from piling up in registers)
      asm volatile("" ::: "memory");
#pragma unroll
      for (int i = 0; i < k; ++i) x[k] -= P[k * 16 + i] * x[i];
    }
#pragma unroll
    for (int k = 1; k < 16; ++k) A[(size_t)(c0 + k) * n + j] = x[k];
  }
  __syncthreads();
}

__global__ __launch_bounds__(kFactorThreads) void k_nd_getrf(const Front *fr, int first,
                                                            double *ar, int *ia, int *info) {
  constexpr int NT = kFactorThreads, NW = NT / 64;
  extern __shared__ double lds[];
  const int fi = first + blockIdx.x;
  const Front f = fr[fi];
  const int n = f.nS;
  const int n16 = (n + 15) & ~15;
  double *A = ar + f.fss;
  double *P = lds;                   // [n16][16] panel
  double *redv = P + (size_t)n16 * 16;
  int *redi = (int *)(redv + NW);    // [NW]
  int *pivl = redi + NW;             // [16] pivot row of each panel column
  int *perm = pivl + 16;             // [n]
  int *zp = perm + n;                // first zero pivot (1-based), 0 if none
  const PanelSlots ps = panel_slots(zp + 1);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < n; i += NT) perm[i] = i;
  if (tid == 0) *zp = 0;
  __syncthreads();
  for (int c0 = 0; c0 < n; c0 += 16) {
    nd_panel<NT>(A, n, c0, P, ps, pivl, perm, zp);
    if (c0 + 16 >= n) break;
    // trailing update A22 -= L21 U12, strips of one row tile x four column tiles
    const int r0 = c0 + 16;
    const int nt = (n - r0 + 15) >> 4, ns = (nt + 3) >> 2;
    for (int st = wv; st < nt * ns; st += NW) {
      const int bi = st / ns, bj = (st - bi * ns) * 4;
      const int rb = r0 + 16 * bi;
      d4 acc[4];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int col = r0 + 16 * (bj + jj) + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = rb + 4 * q + (lane >> 4);
          acc[jj][q] = (row < n && col < n) ? A[(size_t)row * n + col] : 0.0;
        }
      }
      const int arow = rb + (lane & 15);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + (lane >> 4);
        const double a = arow < n ? -P[(arow - c0) * 16 + k] : 0.0;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int col = r0 + 16 * (bj + jj) + (lane & 15);
          const double b = col < n ? A[(size_t)(c0 + k) * n + col] : 0.0;
          acc[jj] = mma(a, b, acc[jj]);
        }
      }
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int col = r0 + 16 * (bj + jj) + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = rb + 4 * q + (lane >> 4);
          if (row < n && col < n) A[(size_t)row * n + col] = acc[jj][q];
        }
      }
    }
    __syncthreads();
  }
  int *permg = ia + f.perm;
  for (int i = tid; i < n; i += NT) permg[i] = perm[i];
  if (tid == 0) info[fi] = *zp;
}

// The same LU for the few large fronts at the top of the tree, in two
// launches per panel: k_nd_panel (one workgroup per front: the panel, its
// exchanges and U12, with the row order and the zero-pivot flag kept in
// global memory between launches) and k_nd_trail (the trailing update of
// every front of the level, one 64 x 64 tile per workgroup).
__global__ __launch_bounds__(kFactorThreads) void k_nd_panel(const Front *fr, int first,
                                                            double *ar, int *ia, int *info,
                                                            int c0) {
  constexpr int NT = kFactorThreads, NW = NT / 64;
  extern __shared__ double lds[];
  const int fi = first + blockIdx.x;
  const Front f = fr[fi];
  const int n = f.nS;
  if (c0 >= n) return;
  const int n16 = (n + 15) & ~15;
  double *P = lds;
  double *redv = P + (size_t)n16 * 16;
  int *redi = (int *)(redv + NW);
  int *pivl = redi + NW;
  int *perm = ia + f.perm;
  const PanelSlots ps = panel_slots(pivl + 16);
  if (c0 == 0) {
    for (int i = threadIdx.x; i < n; i += NT) perm[i] = i;
    if (threadIdx.x == 0) info[fi] = 0;
    __syncthreads();
  }
  nd_panel<NT>(ar + f.fss, n, c0, P, ps, pivl, perm, info + fi);
}

__global__ __launch_bounds__(256) void k_nd_trail(const Front *fr, int first, double *ar,
                                                  int c0) {
  const Front f = fr[first + blockIdx.y];
  const int n = f.nS, r0 = c0 + 16;
  if (r0 >= n) return;
  const int tn = (n - r0 + 63) >> 6;
  if ((int)blockIdx.x >= tn * tn) return;
  const int bi = blockIdx.x / tn, bj = blockIdx.x - bi * tn;
  double *A = ar + f.fss;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wr = wv >> 1, wc = wv & 1;
  const int rb = r0 + 64 * bi + 32 * wr, cb = r0 + 64 * bj + 32 * wc;
  d4 acc[2][2];
#pragma unroll
  for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
    for (int j2 = 0; j2 < 2; ++j2) {
      const int col = cb + 16 * j2 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = rb + 16 * i2 + 4 * q + (lane >> 4);
        acc[i2][j2][q] = (row < n && col < n) ? A[(size_t)row * n + col] : 0.0;
      }
    }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = c0 + 4 * s + (lane >> 4);
    double a[2], b[2];
#pragma unroll
    for (int i2 = 0; i2 < 2; ++i2) {
      const int row = rb + 16 * i2 + (lane & 15);
      a[i2] = row < n ? -A[(size_t)row * n + k] : 0.0;
    }
#pragma unroll
    for (int j2 = 0; j2 < 2; ++j2) {
      const int col = cb + 16 * j2 + (lane & 15);
      b[j2] = col < n ? A[(size_t)k * n + col] : 0.0;
    }
#pragma unroll
    for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
      for (int j2 = 0; j2 < 2; ++j2) acc[i2][j2] = mma(a[i2], b[j2], acc[i2][j2]);
  }
#pragma unroll
  for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
    for (int j2 = 0; j2 < 2; ++j2) {
      const int col = cb + 16 * j2 + (lane & 15);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = rb + 16 * i2 + 4 * q + (lane >> 4);
        if (row < n && col < n) A[(size_t)row * n + col] = acc[i2][j2][q];
      }
    }
}

// ---------------------------------------------------------------------------
// F_ss^{-1} B for 16 right-hand-side columns per workgroup (B = F_se in
// place -> X, or the single column y).  The rows are taken in pivot order
// into LDS; forward (unit L) and back (U) substitution go by 16-row blocks:
// the off-diagonal product of a block is an MFMA contraction split over the
// wavefronts and summed in LDS, the 16 x 16 diagonal solve runs in 16 lanes.
// ---------------------------------------------------------------------------
size_t getrs_lds(int n) {
  const int n16 = (n + 15) & ~15;
  const int nw = kSolveThreads / 64;
  return sizeof(double) * ((size_t)n16 * 16 + (size_t)nw * 256 + 256);
}

__global__ __launch_bounds__(kSolveThreads) void k_nd_getrs(const Front *fr, int first,
                                                           double *ar, const int *ia,
                                                           int single) {
  constexpr int NT = kSolveThreads, NW = NT / 64;
  extern __shared__ double lds[];
  const Front f = fr[first + blockIdx.y];
  const int n = f.nS;
  const int ncol = single ? 1 : f.nE;
  const int j0 = blockIdx.x * 16;
  if (n == 0 || j0 >= ncol) return;
  const int n16 = (n + 15) & ~15, nbk = n16 >> 4;
  double *B = single ? ar + f.y : ar + f.x;
  const int ldb = single ? 1 : f.nE;
  const double *A = ar + f.fss;
  const int *perm = ia + f.perm;
  double *Bs = lds;                         // [n16][16]
  double *red = Bs + (size_t)n16 * 16;      // [NW][256]
  double *Dg = red + NW * 256;              // [16][16] diagonal block
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int e = tid; e < n16 * 16; e += NT) {
    const int r = e >> 4, c = e & 15;
    Bs[e] = (r < n && j0 + c < ncol) ? B[(size_t)perm[r] * ldb + j0 + c] : 0.0;
  }
  // one block step: Bs[rb..rb+15] -= A[rb.., k range] Bs[k range], then the
  // diagonal solve (lower: unit diagonal; upper: divide)
  auto block = [&](int rb, int klo, int khi, bool upper) {
    for (int e = tid; e < 256; e += NT) {
      const int r = rb + (e >> 4), c = rb + (e & 15);
      Dg[e] = (r < n && c < n) ? A[(size_t)r * n + c] : 0.0;
    }
    if (khi > klo) {
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      const int arow = rb + (lane & 15);
      // four contraction steps per round, their loads issued together
      const int s1 = khi >> 2;
      for (int s0 = (klo >> 2) + wv; s0 < s1; s0 += 4 * NW) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int s = s0 + u * NW, kk = 4 * s + (lane >> 4);
          const bool ok = s < s1;
          a[u] = (ok && arow < n && kk < n) ? A[(size_t)arow * n + kk] : 0.0;
          b[u] = ok ? Bs[kk * 16 + (lane & 15)] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = mma(a[u], b[u], acc);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) red[wv * 256 + q * 64 + lane] = acc[q];
    }
    __syncthreads();
    if (khi > klo) {
      for (int e = tid; e < 256; e += NT) {
        double sum = 0.0;
        for (int w2 = 0; w2 < NW; ++w2) sum += red[w2 * 256 + e];
        const int q = e >> 6, ln = e & 63;
        const int r = 4 * q + (ln >> 4), c = ln & 15;
        Bs[(rb + r) * 16 + c] -= sum;
      }
    }
    __syncthreads();
    if (tid < 16) {
      double x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] = Bs[(rb + i) * 16 + tid];
      if (!upper) {
#pragma unroll
        for (int i = 1; i < 16; ++i) {
#pragma unroll
          for (int k = 0; k < i; ++k) x[i] -= Dg[i * 16 + k] * x[k];
        }
      } else {
#pragma unroll
        for (int i = 15; i >= 0; --i) {
          if (rb + i < n) {
#pragma unroll
            for (int k = i + 1; k < 16; ++k) x[i] -= Dg[i * 16 + k] * x[k];
            x[i] /= Dg[i * 16 + i];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) Bs[(rb + i) * 16 + tid] = x[i];
    }
    __syncthreads();
  };
  __syncthreads();
  for (int k = 0; k < nbk; ++k) block(16 * k, 0, 16 * k, false);
  for (int k = nbk - 1; k >= 0; --k) block(16 * k, 16 * (k + 1), n16, true);
  for (int e = tid; e < n16 * 16; e += NT) {
    const int r = e >> 4, c = e & 15;
    if (r < n && j0 + c < ncol) B[(size_t)r * ldb + j0 + c] = Bs[e];
  }
}

// ---------------------------------------------------------------------------
// T_b -= F_es X: 64 x 64 output tiles, four wavefronts of 32 x 32 (2 x 2 MFMA
// tiles), the inner dimension staged through LDS 16 at a time.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_nd_gemm(const Front *fr, int first, double *ar) {
  const Front f = fr[first + blockIdx.y];
  const int M = f.nE, N = f.nE, K = f.nS;
  if (M == 0 || K == 0) return;
  const int tn = (N + 63) >> 6, tm = (M + 63) >> 6;
  if ((int)blockIdx.x >= tm * tn) return;
  const int bi = blockIdx.x / tn, bj = blockIdx.x - bi * tn;
  const double *Am = ar + f.fes;   // M x K
  const double *Bm = ar + f.x;     // K x N
  double *C = ar + f.t;            // M x N
  __shared__ double As[64 * 17];
  __shared__ double Bs[16 * 68];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 16) {
    {
      const int r = tid >> 2, c = (tid & 3) * 4, gr = bi * 64 + r;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int gk = k0 + c + u;
        As[r * 17 + c + u] = (gr < M && gk < K) ? Am[(size_t)gr * K + gk] : 0.0;
      }
    }
    {
      const int r = tid >> 4, c = (tid & 15) * 4, gk = k0 + r;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int gc = bj * 64 + c + u;
        Bs[r * 68 + c + u] = (gk < K && gc < N) ? Bm[(size_t)gk * N + gc] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = 4 * s + (lane >> 4);
      const double a0 = -As[(32 * wr + (lane & 15)) * 17 + kk];
      const double a1 = -As[(32 * wr + 16 + (lane & 15)) * 17 + kk];
      const double b0 = Bs[kk * 68 + 32 * wc + (lane & 15)];
      const double b1 = Bs[kk * 68 + 32 * wc + 16 + (lane & 15)];
      acc[0][0] = mma(a0, b0, acc[0][0]);
      acc[0][1] = mma(a0, b1, acc[0][1]);
      acc[1][0] = mma(a1, b0, acc[1][0]);
      acc[1][1] = mma(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
    for (int j2 = 0; j2 < 2; ++j2)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = bi * 64 + 32 * wr + 16 * i2 + 4 * q + (lane >> 4);
        const int col = bj * 64 + 32 * wc + 16 * j2 + (lane & 15);
        if (row < M && col < N) C[(size_t)row * N + col] += acc[i2][j2][q];
      }
}

// ---------------------------------------------------------------------------
// solve phase
// ---------------------------------------------------------------------------
// r_t = -(w_t + S_t[:, D] g_D) at the slots of the leaf's interface sides
// (the Dirichlet slots are never read); a transformed leaf stores R r_t in
// its edge basis.  One workgroup per leaf.
__global__ __launch_bounds__(128) void k_nd_leaf_rhs(const LeafD *ld, const double *S,
                                                     const double *w, const double *g,
                                                     const double *tab, double *rl, double *ar) {
  __shared__ double rf[4 * HPS_P_MAX];
  const LeafD &L = ld[blockIdx.x];
  const int m = L.m, nb = 4 * m;
  for (int s = threadIdx.x; s < nb; s += 128) {
    const int side = s / m;
    double v = 0.0;
    if (!L.side[side].dir) {
      v = w ? w[L.b_off + s] : 0.0;
      const double *row = S + L.s_off + (size_t)s * nb;
      for (int d = 0; d < 4; ++d) {
        if (!L.side[d].dir) continue;
        for (int k = d * m; k < d * m + m; ++k) v += row[k] * g[L.b_off + k];
      }
      v = -v;
    }
    if (L.t_off < 0) rl[L.b_off + s] = v;
    else rf[s] = v;
  }
  if (L.t_off < 0) return;
  __syncthreads();
  for (int a = threadIdx.x; a < L.ne; a += 128) {
    int s, i;
    edge_basis(L, a, s, i);
    const Side sd = L.side[s];
    double v;
    if (sd.R < 0) {
      v = rf[s * m + i];
    } else {
      v = 0.0;
      for (int k = 0; k < m; ++k) v += tab[sd.R + i * m + k] * rf[s * m + k];
    }
    ar[L.r_off + a] = v;
  }
}

// y = r_s and r_b = r_e, scattered from the halves' reduced right-hand sides
__global__ __launch_bounds__(256) void k_nd_front_rhs(const Front *fr, int first, double *ar,
                                                      const int *ia, const double *rl) {
  const Front f = fr[first + blockIdx.x];
  const int n = f.nS + f.nE;
  const double *ra = child_r(f, true, ar, rl);
  const double *rc = child_r(f, false, ar, rl);
  const int *ma = ia + f.map, *mc = ma + n;
  for (int i = threadIdx.x; i < n; i += 256) {
    double v = 0.0;
    if (ma[i] >= 0) v = ra[ma[i]];
    if (mc[i] >= 0) v += rc[mc[i]];
    if (i < f.nS) ar[f.y + i] = v;
    else ar[f.r + (i - f.nS)] = v;
  }
}

__global__ __launch_bounds__(256) void k_nd_gemv_r(const Front *fr, int first, double *ar) {
  const Front f = fr[first + blockIdx.y];
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= f.nE) return;
  const double *a = ar + f.fes + (size_t)row * f.nS;
  const double *y = ar + f.y;
  double s = 0.0;
  for (int k = lane; k < f.nS; k += 64) s += a[k] * y[k];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) ar[f.r + row] -= s;
}

// u_s = y - X u_E (u: every edge node of the grid), one wavefront per row
__global__ __launch_bounds__(256) void k_nd_down(const Front *fr, int first, const double *ar,
                                                 const int *ia, double *u) {
  const Front f = fr[first + blockIdx.y];
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= f.nS) return;
  const int *gid = ia + f.gid;
  const double *x = ar + f.x + (size_t)row * f.nE;
  double s = 0.0;
  for (int k = lane; k < f.nE; k += 64) s += x[k] * u[gid[f.nS + k]];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) u[gid[row]] = ar[f.y + row] - s;
}

// ub: solved interface values, g on the outer boundary
// ub: interface values (interpolated to the leaf's nodes where its edge
// carries a lower order's nodes), g on the outer boundary.  One workgroup
// per leaf.
__global__ __launch_bounds__(128) void k_nd_output(const LeafD *ld, const double *u,
                                                   const double *g, const double *tab,
                                                   double *ub) {
  const LeafD &L = ld[blockIdx.x];
  const int m = L.m, nb = 4 * m;
  for (int s = threadIdx.x; s < nb; s += 128) {
    const int side = s / m, k = s - side * m;
    const Side sd = L.side[side];
    double v;
    if (sd.dir) {
      v = g[L.b_off + s];
    } else if (sd.P < 0) {
      v = u[sd.node0 + k];
    } else {
      v = 0.0;
      for (int j = 0; j < sd.me; ++j) v += tab[sd.P + k * sd.me + j] * u[sd.node0 + j];
    }
    ub[L.b_off + s] = v;
  }
}

// ---------------------------------------------------------------------------
// host planning
// ---------------------------------------------------------------------------
struct Plan {
  int nx = 0, ny = 0, L = 0;
  std::vector<Front> fronts;      // ordered by level
  std::vector<int> level_first;   // fronts of level l: [level_first[l], level_first[l+1])
  std::vector<int> level_max_s, level_max_e;
  std::vector<int> ints;          // int arena (maps, node ids; pivot orders left 0)
  std::vector<LeafD> leaves;
  std::vector<int> tlist;         // leaves taken to the edge basis
  int t_max_m = 0, t_max_ne = 0;
  std::vector<double> tab;        // interpolation matrices
  size_t ndouble = 0;
  size_t nslot = 0;               // extent of the slot arrays (w, g, ub)
  int max_sep = 0;
  double flop = 0.0;
  int nnode = 0;                  // edge nodes of the grid (Dirichlet included)
};

// M [m_to][m_from]: values at the interior Chebyshev extreme points of order
// m_to + 2 of the polynomial through values at those of order m_from + 2.
void interp_matrix(int m_from, int m_to, double *M) {
  const long double pi = 3.141592653589793238462643383279502884L;
  auto pts = [&](int m) {
    std::vector<long double> t(m);
    const int n = m + 1;
    for (int k = 1; k <= m; ++k) t[k - 1] = std::sin(pi * (long double)(2 * k - n) / (2.0L * n));
    return t;
  };
  const std::vector<long double> s = pts(m_from), t = pts(m_to);
  for (int i = 0; i < m_to; ++i)
    for (int k = 0; k < m_from; ++k) {
      long double v = 1.0L;
      for (int q = 0; q < m_from; ++q)
        if (q != k) v *= (t[i] - s[q]) / (s[k] - s[q]);
      M[(size_t)i * m_from + k] = (double)v;
    }
}

struct BoxOut {
  int front = -1;              // -1: a leaf
  int leaf = -1;
  int level = 0;
  std::vector<int> E;          // unknown boundary nodes
  std::vector<int> pos;        // row of each in the box's Schur complement
};

struct FrontH {
  int nS = 0, nE = 0, level = 0;
  int childA = 0, childC = 0;  // >= 0 front index, < 0: -(leaf+1)
  std::vector<int> map_a, map_c, gid;
};

struct Planner {
  int nx, ny;
  const std::vector<LeafD> *leaves;
  std::vector<FrontH> fronts;
  int max_sep = 0;

  BoxOut build(int x0, int x1, int y0, int y1) {
    BoxOut out;
    if (x1 - x0 == 1 && y1 - y0 == 1) {
      out.leaf = x0 + nx * y0;
      const LeafD &L = (*leaves)[out.leaf];
      int run = 0;
      for (int s = 0; s < 4; ++s) {
        const Side &sd = L.side[s];
        if (sd.dir) continue;
        for (int k = 0; k < sd.me; ++k) {
          out.E.push_back(sd.node0 + k);
          out.pos.push_back(L.t_off >= 0 ? run + k : s * L.m + k);
        }
        run += sd.me;
      }
      return out;
    }
    BoxOut a, c;
    if (x1 - x0 >= y1 - y0) {
      const int mid = x0 + (x1 - x0) / 2;
      a = build(x0, mid, y0, y1);
      c = build(mid, x1, y0, y1);
    } else {
      const int mid = y0 + (y1 - y0) / 2;
      a = build(x0, x1, y0, mid);
      c = build(x0, x1, mid, y1);
    }
    std::unordered_map<int, int> in_c;
    in_c.reserve(c.E.size() * 2);
    for (size_t k = 0; k < c.E.size(); ++k) in_c[c.E[k]] = (int)k;
    std::vector<char> shared_c(c.E.size(), 0);
    FrontH fh;
    std::vector<int> sep_a, sep_c, ext_a, ext_c;   // indices into a.E / c.E
    for (size_t k = 0; k < a.E.size(); ++k) {
      auto it = in_c.find(a.E[k]);
      if (it != in_c.end()) {
        sep_a.push_back((int)k);
        sep_c.push_back(it->second);
        shared_c[it->second] = 1;
      } else {
        ext_a.push_back((int)k);
      }
    }
    for (size_t k = 0; k < c.E.size(); ++k)
      if (!shared_c[k]) ext_c.push_back((int)k);
    fh.nS = (int)sep_a.size();
    fh.nE = (int)(ext_a.size() + ext_c.size());
    const int n = fh.nS + fh.nE;
    fh.map_a.assign(n, -1);
    fh.map_c.assign(n, -1);
    fh.gid.resize(n);
    for (int k = 0; k < fh.nS; ++k) {
      fh.map_a[k] = a.pos[sep_a[k]];
      fh.map_c[k] = c.pos[sep_c[k]];
      fh.gid[k] = a.E[sep_a[k]];
    }
    int o = fh.nS;
    for (int k : ext_a) {
      fh.map_a[o] = a.pos[k];
      fh.gid[o] = a.E[k];
      out.E.push_back(a.E[k]);
      ++o;
    }
    for (int k : ext_c) {
      fh.map_c[o] = c.pos[k];
      fh.gid[o] = c.E[k];
      out.E.push_back(c.E[k]);
      ++o;
    }
    out.pos.resize(out.E.size());
    for (size_t k = 0; k < out.pos.size(); ++k) out.pos[k] = (int)k;
    fh.childA = a.front >= 0 ? a.front : -(a.leaf + 1);
    fh.childC = c.front >= 0 ? c.front : -(c.leaf + 1);
    fh.level = 1 + std::max(a.level, c.level);
    max_sep = std::max(max_sep, fh.nS);
    out.front = (int)fronts.size();
    out.level = fh.level;
    fronts.push_back(std::move(fh));
    return out;
  }
};

auto align32 = [](size_t v) { return (v + 31) & ~(size_t)31; };

// Edges of the grid (vertical: line ix = 0..nx, row iy; then horizontal:
// column ix, line iy = 0..ny), their node counts (the lower order of the two
// leaves that share it; an outer edge keeps its leaf's), the leaves' sides
// and interpolations.  Offsets s_off / b_off (may be null: leaf-major with
// one order) place each leaf's S and slots in the caller's arrays.
hps_status make_leaves(int nx, int ny, const int *orders, const long long *s_off,
                       const long long *b_off, Plan &pl) {
  const int L = nx * ny;
  const int nv = (nx + 1) * ny, nedge = nv + nx * (ny + 1);
  std::vector<int> me(nedge, INT_MAX), owners(nedge, 0);
  auto edges_of = [&](int t, int e[4]) {
    const int ix = t % nx, iy = t / nx;
    e[0] = ix + (nx + 1) * iy;
    e[1] = ix + 1 + (nx + 1) * iy;
    e[2] = nv + ix + nx * iy;
    e[3] = nv + ix + nx * (iy + 1);
  };
  for (int t = 0; t < L; ++t) {
    if (orders[t] < HPS_P_MIN || orders[t] > HPS_P_MAX) return HPS_ERR_INVALID;
    if ((s_off && s_off[t] < 0) || (b_off && b_off[t] < 0)) return HPS_ERR_INVALID;
    int e[4];
    edges_of(t, e);
    for (int s = 0; s < 4; ++s) {
      me[e[s]] = std::min(me[e[s]], orders[t] - 2);
      owners[e[s]]++;
    }
  }
  std::vector<int> node0(nedge + 1, 0);
  for (int e = 0; e < nedge; ++e) node0[e + 1] = node0[e] + me[e];
  pl.nnode = node0[nedge];
  std::map<std::pair<int, int>, int> tabs;   // (m_from, m_to) -> offset
  auto table = [&](int m_from, int m_to) {
    auto it = tabs.find({m_from, m_to});
    if (it != tabs.end()) return it->second;
    const int off = (int)pl.tab.size();
    pl.tab.resize(pl.tab.size() + (size_t)m_from * m_to);
    interp_matrix(m_from, m_to, pl.tab.data() + off);
    tabs[{m_from, m_to}] = off;
    return off;
  };
  pl.leaves.assign(L, LeafD{});
  long long s_run = 0, b_run = 0;
  for (int t = 0; t < L; ++t) {
    LeafD &d = pl.leaves[t];
    d.m = orders[t] - 2;
    const int nb = 4 * d.m;
    d.s_off = s_off ? s_off[t] : s_run;
    d.b_off = b_off ? b_off[t] : b_run;
    s_run += (long long)nb * nb;
    b_run += nb;
    pl.nslot = std::max(pl.nslot, (size_t)(d.b_off + nb));
    int e[4];
    edges_of(t, e);
    d.ne = 0;
    bool transformed = false;
    for (int s = 0; s < 4; ++s) {
      Side &sd = d.side[s];
      sd.node0 = node0[e[s]];
      sd.me = me[e[s]];
      sd.dir = owners[e[s]] == 1;
      sd.P = sd.R = -1;
      if (!sd.dir) {
        d.ne += sd.me;
        if (sd.me < d.m) {
          transformed = true;
          sd.P = table(sd.me, d.m);   // [m][me]
          sd.R = table(d.m, sd.me);   // [me][m]
        }
      }
    }
    d.t_off = d.r_off = transformed ? 0 : -1;
    if (transformed) {
      pl.tlist.push_back(t);
      pl.t_max_m = std::max(pl.t_max_m, d.m);
      pl.t_max_ne = std::max(pl.t_max_ne, d.ne);
    }
  }
  return HPS_OK;
}

hps_status make_plan(int nx, int ny, const int *orders, const long long *s_off,
                     const long long *b_off, Plan &pl) {
  if (!orders || nx < 1 || ny < 1) return HPS_ERR_INVALID;
  if ((long long)nx * ny > (1 << 22)) return HPS_ERR_INVALID;
  pl.nx = nx;
  pl.ny = ny;
  pl.L = nx * ny;
  const hps_status st = make_leaves(nx, ny, orders, s_off, b_off, pl);
  if (st != HPS_OK) return st;
  Planner P{nx, ny, &pl.leaves, {}, 0};
  P.build(0, nx, 0, ny);
  pl.max_sep = P.max_sep;
  if (P.max_sep > kMaxSep) return HPS_ERR_INVALID;
  const int nf = (int)P.fronts.size();
  int nlev = 0;
  for (const auto &f : P.fronts) nlev = std::max(nlev, f.level);
  // order by level (stable), then lay out the arenas in that order
  std::vector<int> order(nf), where(nf);
  for (int k = 0; k < nf; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return P.fronts[a].level < P.fronts[b].level; });
  for (int k = 0; k < nf; ++k) where[order[k]] = k;
  pl.fronts.assign(nf, Front{});
  pl.level_first.assign(nlev + 2, nf);
  pl.level_max_s.assign(nlev + 1, 0);
  pl.level_max_e.assign(nlev + 1, 0);
  size_t od = 0;
  // level_first[l]: first front (in level order) whose level is at least l
  for (int l = 1, k = 0; l <= nlev + 1; ++l) {
    while (k < nf && P.fronts[order[k]].level < l) ++k;
    pl.level_first[l] = k;
  }
  for (int k = 0; k < nf; ++k) {
    const FrontH &h = P.fronts[order[k]];
    Front &f = pl.fronts[k];
    const size_t s = h.nS, e = h.nE;
    f.nS = h.nS;
    f.nE = h.nE;
    f.fss = (long long)od; od = align32(od + s * s);
    f.x = (long long)od;   od = align32(od + s * e);
    f.fes = (long long)od; od = align32(od + e * s);
    f.t = (long long)od;   od = align32(od + e * e);
    f.y = (long long)od;   od = align32(od + s);
    f.r = (long long)od;   od = align32(od + e);
    f.map = (int)pl.ints.size();
    pl.ints.insert(pl.ints.end(), h.map_a.begin(), h.map_a.end());
    pl.ints.insert(pl.ints.end(), h.map_c.begin(), h.map_c.end());
    f.gid = (int)pl.ints.size();
    pl.ints.insert(pl.ints.end(), h.gid.begin(), h.gid.end());
    f.perm = (int)pl.ints.size();
    pl.ints.insert(pl.ints.end(), (size_t)h.nS, 0);
    pl.level_max_s[h.level] = std::max(pl.level_max_s[h.level], h.nS);
    pl.level_max_e[h.level] = std::max(pl.level_max_e[h.level], h.nE);
    pl.flop += (2.0 / 3.0) * s * s * s + 2.0 * s * s * e + 2.0 * e * e * s;
  }
  // transformed leaves: R S P and R r in the arena
  for (int t : pl.tlist) {
    LeafD &d = pl.leaves[t];
    d.t_off = (long long)od; od = align32(od + (size_t)d.ne * d.ne);
    d.r_off = (long long)od; od = align32(od + (size_t)d.ne);
  }
  // children: fronts and transformed leaves in the arena, other leaves in S
  for (int k = 0; k < nf; ++k) {
    const FrontH &h = P.fronts[order[k]];
    Front &f = pl.fronts[k];
    auto child = [&](int c, long long &tOff, long long &rOff, int &kind, int &ld) {
      if (c < 0) {
        const LeafD &d = pl.leaves[-c - 1];
        if (d.t_off >= 0) {
          kind = 0;
          tOff = d.t_off;
          rOff = d.r_off;
          ld = d.ne;
        } else {
          kind = 1;
          tOff = d.s_off;
          rOff = d.b_off;
          ld = 4 * d.m;
        }
      } else {
        const Front &cf = pl.fronts[where[c]];
        kind = 0;
        tOff = cf.t;
        rOff = cf.r;
        ld = cf.nE;
      }
    };
    child(h.childA, f.ca, f.ra, f.ka, f.lda);
    child(h.childC, f.cc, f.rc, f.kc, f.ldc);
  }
  pl.ndouble = od;
  return HPS_OK;
}

size_t plan_bytes(const Plan &pl) {
  return pl.ndouble * sizeof(double) + pl.ints.size() * sizeof(int) +
         pl.fronts.size() * (sizeof(Front) + sizeof(int)) + pl.leaves.size() * sizeof(LeafD) +
         pl.tlist.size() * sizeof(int) + pl.tab.size() * sizeof(double) +
         (pl.nslot + (size_t)pl.nnode) * sizeof(double);
}

template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

hps_status from_hip(hipError_t e) {
  if (e == hipSuccess) return HPS_OK;
  if (e == hipErrorOutOfMemory) return HPS_ERR_OOM;
  return HPS_ERR_HIP;
}

}  // namespace

struct hps_iface {
  hipStream_t stream = nullptr;
  Plan plan;
  Front *d_front = nullptr;
  LeafD *d_leaf = nullptr;
  int *d_tlist = nullptr;
  double *d_tab = nullptr;
  double *d_ar = nullptr;
  int *d_ia = nullptr;
  int *d_info = nullptr;
  double *d_rl = nullptr;   // leaf right-hand sides, in the slot layout
  double *d_u = nullptr;    // every edge node's value
};

namespace {

hps_status plan_checked(int nx, int ny, const int *orders, const long long *s_off,
                        const long long *b_off, Plan &pl) {
  try {
    return make_plan(nx, ny, orders, s_off, b_off, pl);
  } catch (...) {
    return HPS_ERR_OOM;
  }
}

std::vector<int> uniform_orders(int p, int nx, int ny) {
  return std::vector<int>((size_t)std::max(nx, 0) * std::max(ny, 0), p);
}

hps_status report(const Plan &pl, int *nfront, int *levels, int *max_sep, double *factor_flop,
                  size_t *bytes) {
  if (nfront) *nfront = (int)pl.fronts.size();
  if (levels) *levels = (int)pl.level_first.size() - 2;
  if (max_sep) *max_sep = pl.max_sep;
  if (factor_flop) *factor_flop = pl.flop;
  if (bytes) *bytes = plan_bytes(pl);
  return HPS_OK;
}

}  // namespace

extern "C" {

hps_status hps_iface_plan(int p, int nx, int ny, int *nfront, int *levels, int *max_sep,
                          double *factor_flop, size_t *bytes) {
  if (nx < 1 || ny < 1) return HPS_ERR_INVALID;
  Plan pl;
  const std::vector<int> o = uniform_orders(p, nx, ny);
  const hps_status st = plan_checked(nx, ny, o.data(), nullptr, nullptr, pl);
  if (st != HPS_OK) return st;
  return report(pl, nfront, levels, max_sep, factor_flop, bytes);
}

hps_status hps_iface_plan_orders(int nx, int ny, const int *orders, int *nfront, int *levels,
                                 int *max_sep, double *factor_flop, size_t *bytes) {
  Plan pl;
  const hps_status st = plan_checked(nx, ny, orders, nullptr, nullptr, pl);
  if (st != HPS_OK) return st;
  return report(pl, nfront, levels, max_sep, factor_flop, bytes);
}

hps_status hps_iface_plan_fronts(int p, int nx, int ny, int *nS, int *nE, int *level) {
  if (nx < 1 || ny < 1) return HPS_ERR_INVALID;
  Plan pl;
  const std::vector<int> o = uniform_orders(p, nx, ny);
  const hps_status st = plan_checked(nx, ny, o.data(), nullptr, nullptr, pl);
  if (st != HPS_OK) return st;
  const int nlev = (int)pl.level_first.size() - 2;
  for (int l = 1; l <= nlev; ++l)
    for (int k = pl.level_first[l]; k < pl.level_first[l + 1]; ++k) {
      if (nS) nS[k] = pl.fronts[k].nS;
      if (nE) nE[k] = pl.fronts[k].nE;
      if (level) level[k] = l;
    }
  return HPS_OK;
}

hps_status hps_iface_create_orders(hps_ctx *ctx, int nx, int ny, const int *orders,
                                   const long long *s_off, const long long *b_off,
                                   hps_iface **out) {
  if (!ctx || !out) return HPS_ERR_INVALID;
  *out = nullptr;
  hps_iface *it = new (std::nothrow) hps_iface;
  if (!it) return HPS_ERR_OOM;
  const hps_status st = plan_checked(nx, ny, orders, s_off, b_off, it->plan);
  if (st != HPS_OK) {
    delete it;
    return st;
  }
  it->stream = hps::ctx_stream(ctx);
  const Plan &pl = it->plan;
  const size_t nf = pl.fronts.size();
  hipError_t e = hipSuccess;
  auto alloc = [&](void **ptr, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMalloc(ptr, bytes);
  };
  auto upload = [&](void *dst, const void *src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  };
  alloc((void **)&it->d_front, nf * sizeof(Front));
  alloc((void **)&it->d_leaf, pl.leaves.size() * sizeof(LeafD));
  alloc((void **)&it->d_tlist, pl.tlist.size() * sizeof(int));
  alloc((void **)&it->d_tab, pl.tab.size() * sizeof(double));
  alloc((void **)&it->d_ar, pl.ndouble * sizeof(double));
  alloc((void **)&it->d_ia, pl.ints.size() * sizeof(int));
  alloc((void **)&it->d_info, (nf + 1) * sizeof(int));
  alloc((void **)&it->d_rl, pl.nslot * sizeof(double));
  alloc((void **)&it->d_u, (size_t)pl.nnode * sizeof(double));
  upload(it->d_front, pl.fronts.data(), nf * sizeof(Front));
  upload(it->d_leaf, pl.leaves.data(), pl.leaves.size() * sizeof(LeafD));
  upload(it->d_tlist, pl.tlist.data(), pl.tlist.size() * sizeof(int));
  upload(it->d_tab, pl.tab.data(), pl.tab.size() * sizeof(double));
  upload(it->d_ia, pl.ints.data(), pl.ints.size() * sizeof(int));
  if (e == hipSuccess) e = allow_lds(k_nd_getrf, getrf_lds(kMaxSep));
  if (e == hipSuccess) e = allow_lds(k_nd_panel, getrf_lds(kMaxSep));
  if (e == hipSuccess) e = allow_lds(k_nd_getrs, getrs_lds(kMaxSep));
  if (e == hipSuccess) e = allow_lds(k_nd_leaf_transform, transform_lds(HPS_P_MAX - 2, 4 * (HPS_P_MAX - 2)));
  if (e != hipSuccess) {
    hps_iface_destroy(it);
    return from_hip(e);
  }
  *out = it;
  return HPS_OK;
}

hps_status hps_iface_create(hps_ctx *ctx, int p, int nx, int ny, hps_iface **out) {
  if (!ctx || !out || nx < 1 || ny < 1) return HPS_ERR_INVALID;
  const std::vector<int> o = uniform_orders(p, nx, ny);
  return hps_iface_create_orders(ctx, nx, ny, o.data(), nullptr, nullptr, out);
}

hps_status hps_iface_factor(hps_iface *it, const double *S, int *info, int flags) {
  if (!it || !S) return HPS_ERR_INVALID;
  const Plan &pl = it->plan;
  const hipStream_t st = it->stream;
  if (!pl.tlist.empty())
    k_nd_leaf_transform<<<(int)pl.tlist.size(), 256, transform_lds(pl.t_max_m, pl.t_max_ne),
                          st>>>(it->d_leaf, it->d_tlist, S, it->d_tab, it->d_ar);
  const int nlev = (int)pl.level_first.size() - 2;
  for (int l = 1; l <= nlev; ++l) {
    const int first = pl.level_first[l], cnt = pl.level_first[l + 1] - first;
    if (cnt <= 0) continue;
    const int ms = pl.level_max_s[l], me = pl.level_max_e[l];
    const long long nn = (long long)(ms + me) * (ms + me);
    const int gx = (int)std::min<long long>((nn + 255) / 256, 4096);
    k_nd_front<<<dim3(gx, cnt), 256, 0, st>>>(it->d_front, first, it->d_ar, it->d_ia, S);
    if (ms >= kSplitLU) {
      // few large fronts: the trailing updates spread over the whole GPU
      for (int c0 = 0; c0 < ms; c0 += 16) {
        k_nd_panel<<<cnt, kFactorThreads, getrf_lds(ms), st>>>(it->d_front, first, it->d_ar,
                                                                it->d_ia, it->d_info, c0);
        if (c0 + 16 < ms) {
          const int tn = (ms - c0 - 16 + 63) / 64;
          k_nd_trail<<<dim3(tn * tn, cnt), 256, 0, st>>>(it->d_front, first, it->d_ar, c0);
        }
      }
    } else {
      k_nd_getrf<<<cnt, kFactorThreads, getrf_lds(ms), st>>>(it->d_front, first, it->d_ar,
                                                              it->d_ia, it->d_info);
    }
    if (me > 0) {
      k_nd_getrs<<<dim3((me + 15) / 16, cnt), kSolveThreads, getrs_lds(ms), st>>>(
          it->d_front, first, it->d_ar, it->d_ia, 0);
      const int tiles = ((me + 63) / 64) * ((me + 63) / 64);
      k_nd_gemm<<<dim3(tiles, cnt), 256, 0, st>>>(it->d_front, first, it->d_ar);
    }
  }
  hipError_t e = hipGetLastError();
  const int nf = (int)pl.fronts.size();
  if (e == hipSuccess && info && nf)
    e = hipMemcpyAsync(info, it->d_info, nf * sizeof(int), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && (flags & HPS_SYNC)) {
    e = hipStreamSynchronize(st);
    if (e == hipSuccess && nf) {
      std::vector<int> h(nf);
      e = hipMemcpy(h.data(), it->d_info, nf * sizeof(int), hipMemcpyDeviceToHost);
      if (e == hipSuccess)
        for (int v : h)
          if (v != 0) return HPS_ERR_SINGULAR;
    }
  }
  return from_hip(e);
}

hps_status hps_iface_solve(hps_iface *it, const double *S, const double *w, const double *g,
                           double *ub, int flags) {
  if (!it || !S || !g || !ub) return HPS_ERR_INVALID;
  const Plan &pl = it->plan;
  const hipStream_t st = it->stream;
  const int nlev = (int)pl.level_first.size() - 2;
  k_nd_leaf_rhs<<<pl.L, 128, 0, st>>>(it->d_leaf, S, w, g, it->d_tab, it->d_rl, it->d_ar);
  for (int l = 1; l <= nlev; ++l) {
    const int first = pl.level_first[l], cnt = pl.level_first[l + 1] - first;
    if (cnt <= 0) continue;
    const int ms = pl.level_max_s[l], me = pl.level_max_e[l];
    k_nd_front_rhs<<<cnt, 256, 0, st>>>(it->d_front, first, it->d_ar, it->d_ia, it->d_rl);
    k_nd_getrs<<<dim3(1, cnt), kSolveThreads, getrs_lds(ms), st>>>(it->d_front, first,
                                                                  it->d_ar, it->d_ia, 1);
    if (me > 0)
      k_nd_gemv_r<<<dim3((me + 3) / 4, cnt), 256, 0, st>>>(it->d_front, first, it->d_ar);
  }
  for (int l = nlev; l >= 1; --l) {
    const int first = pl.level_first[l], cnt = pl.level_first[l + 1] - first;
    if (cnt <= 0) continue;
    const int ms = pl.level_max_s[l];
    k_nd_down<<<dim3((ms + 3) / 4, cnt), 256, 0, st>>>(it->d_front, first, it->d_ar, it->d_ia,
                                                       it->d_u);
  }
  k_nd_output<<<pl.L, 128, 0, st>>>(it->d_leaf, it->d_u, g, it->d_tab, ub);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && (flags & HPS_SYNC)) e = hipStreamSynchronize(st);
  return from_hip(e);
}

hps_status hps_iface_destroy(hps_iface *it) {
  if (!it) return HPS_OK;
  hipError_t first = hipSuccess;
  auto rel = [&](void *p) {
    if (!p) return;
    const hipError_t e = hipFree(p);
    if (first == hipSuccess) first = e;
  };
  rel(it->d_front);
  rel(it->d_leaf);
  rel(it->d_tlist);
  rel(it->d_tab);
  rel(it->d_ar);
  rel(it->d_ia);
  rel(it->d_info);
  rel(it->d_rl);
  rel(it->d_u);
  delete it;
  return from_hip(first);
}

}  // extern "C"
