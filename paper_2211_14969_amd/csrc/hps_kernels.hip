// HIP kernels for batched HPS leaf condensation on gfx950 (CDNA4).
//
// Per leaf the interior block A_ii (ni x ni) and the right-hand sides (the
// nb columns of A_ib, and f_i when given) are formed on the device into one
// work matrix  W = [A_ii | rhs]  of R x (16*CT) entries, R = ni rounded up to
// 16 (padding rows/columns carry an identity block so they decouple).
// W is stored tile-major in 16 x 16 tiles whose element order is the
// accumulator layout of the 16x16x4 MFMA instruction of the working
// precision, so a wavefront loads or stores a whole tile with four fully
// coalesced 512-byte accesses.
//
// Elimination (the leaf operations of Sec. 2: an LU factorisation and matrix
// products on every leaf) is a blocked LU with partial pivoting over panels of
// 16 columns.  Rows are never swapped: a pivot row is retired in place and
// its step recorded (rstep), so the row permutation is implicit.  The panel
// is factored in LDS (wavefront + workgroup argmax), the pivot rows of the
// trailing columns become U12 = L11^{-1} A12, and every remaining active row
// tile is updated with MFMA, C -= L21 * U12.  Because the right-hand sides
// are columns of W, the forward elimination of A_ib happens in the same
// pass; a blocked back substitution (MFMA updates again) then yields
// X = A_ii^{-1} A_ib and h = A_ii^{-1} f_i.
//
// The pivoting follows LAPACK getrf: the largest magnitude in the column
// among the rows not yet retired, ties to the lowest row index.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <type_traits>
#include <utility>

#include "hps_internal.h"

namespace hps {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  using acc = d4;
  __device__ static __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
// FP32 work matrices take their tile products on the FP64 MFMA: the FP32
// operands are exact in FP64, so every product is exact and accumulation is
// FP64 before rounding back to FP32 storage.  (The FP32 16x16x4 instruction
// is true FP32 arithmetic, but its FP32 accumulation over the long inner
// dimensions of the larger orders left leaves that FP64 refinement could
// not serve.)
template <>
struct Mfma<float> {
  using acc = d4;
  __device__ static __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64((double)a, (double)b, c, 0, 0, 0);
  }
};

// Element (r, c) of a tile-major work matrix with CT column tiles.  Inside a
// 16 x 16 tile the 256 elements are ordered as the accumulator registers of
// the FP64 16x16x4 MFMA instruction, which both precisions use: element
// q*64 + lane holds accumulator register q of that lane, i.e. row r in
// register r/4 of lanes 16*(r%4) .. +15, column = lane%16 -- plain
// row-major order within the tile.  (The FP32 instruction's accumulators are
// ordered differently: row r in register r%4 of lanes 16*(r/4) .. +15.)
// The A (16x4) and B (4x16) operand layouts agree: A[i][k] and B[k][j] sit in
// lane i + 16k and lane j + 16k.
template <typename T>
struct Tile;
template <>
struct Tile<double> {
  __device__ static __forceinline__ int inner(int r, int c) { return ((r & 15) << 4) + (c & 15); }
  __device__ static __forceinline__ int crow(int q, int lane) { return 4 * q + (lane >> 4); }
  __device__ static __forceinline__ void rc(int w, int &r, int &c) {
    r = w >> 4;
    c = w & 15;
  }
};
template <>
struct Tile<float> : Tile<double> {};   // FP64 MFMA accumulator order

template <typename T>
__device__ __forceinline__ size_t tix(int r, int c, int CT) {
  return ((size_t)((r >> 4) * CT + (c >> 4)) << 8) + Tile<T>::inner(r, c);
}

// Leaf handled by this block (false: the block has nothing to do).
__device__ __forceinline__ bool resolve_leaf(const Sel &sel, int &leaf) {
  leaf = blockIdx.x;
  if (!sel.list) return true;
  const int slot = sel.slot0 + (int)blockIdx.x;
  if (slot >= *sel.count) return false;
  leaf = sel.list[slot];
  return true;
}

// Elements of a leaf's work matrix W, and of its slot in the workspace: W
// followed by one 16 x 16 tile per panel (the left-looking factorisation
// keeps each panel's L11^{-1} there).
__device__ __forceinline__ size_t work_elems(const Geom &g) {
  return (size_t)g.RT * g.CT * 256;
}
__device__ __forceinline__ size_t leaf_stride(const Geom &g) {
  return (size_t)leaf_tiles(g) * 256;
}

// Boundary slot b -> grid node (k, l):  W, E, S, N, each p-2 nodes.
__device__ __forceinline__ void bnode(int b, int m, int p, int &k, int &l) {
  const int s = b / m, t = b - s * m + 1;
  if (s == 0) { k = 0; l = t; }
  else if (s == 1) { k = p - 1; l = t; }
  else if (s == 2) { k = t; l = 0; }
  else { k = t; l = p - 1; }
}

struct LeafScale {
  double sx, sy;  // 2/hx, 2/hy
};

__device__ __forceinline__ LeafScale leaf_scale(const Geom &g, int leaf) {
  const double *b = g.box + 4 * (size_t)leaf;
  LeafScale s;
  s.sx = 2.0 / (b[1] - b[0]);
  s.sy = 2.0 / (b[3] - b[2]);
  return s;
}

// Entry of the collocated operator in the row of interior node (i, j) and
// the column of node (k, l):
//   -(a11 d11 + c1 d1) along x1, -(a22 d22 + c2 d2) along x2, -k2b on the
// diagonal, with d1 = (2/hx) D, d11 = (2/hx)^2 D^2 (likewise in x2), and
// with a mixed term -2 a12 d1x[i][k] d1y[j][l] at every node (k, l).
__device__ __forceinline__ double opval(const Geom &g, const double *sD,
                                        const double *sD2, LeafScale sc,
                                        size_t nbase, int i, int j, int k, int l) {
  const int p = g.p;
  const size_t n = nbase + i + (size_t)p * j;
  double v = 0.0;
  if (l == j) {
    const double a = g.a11 ? g.a11[n] : 1.0;
    const double c = g.c1 ? g.c1[n] : 0.0;
    v -= a * (sc.sx * sc.sx) * sD2[i * p + k] + c * sc.sx * sD[i * p + k];
  }
  if (k == i) {
    const double a = g.a22 ? g.a22[n] : 1.0;
    const double c = g.c2 ? g.c2[n] : 0.0;
    v -= a * (sc.sy * sc.sy) * sD2[j * p + l] + c * sc.sy * sD[j * p + l];
  }
  if (k == i && l == j && g.k2b) v -= g.k2b[n];
  if (g.a12) v -= 2.0 * g.a12[n] * (sc.sx * sD[i * p + k]) * (sc.sy * sD[j * p + l]);
  return v;
}

// Entry of A_ib: the row of interior node (i, j), the column of boundary slot
// b.  With a mixed term the row also reaches the leaf corners, which carry no
// unknown: each corner value is the mean of the degree-(p-3) extrapolants
// along its two edges (weights E[0] to an edge's low end, E[1] to its high
// end), so an edge slot collects half of each of its edge's two corners.
__device__ __forceinline__ double aib_elem(const Geom &g, const double *sD, const double *sD2,
                                           LeafScale sc, size_t nbase, int i, int j, int b) {
  const int p = g.p, m = g.m;
  int k, l;
  bnode(b, m, p, k, l);
  double v = opval(g, sD, sD2, sc, nbase, i, j, k, l);
  if (g.a12) {
    const int s = b / m, q = b - s * m;
    int k0, l0, k1, l1;   // the edge's corners at its low and high ends
    if (s < 2) {          // W / E: along x2
      k0 = k1 = (s == 0) ? 0 : p - 1;
      l0 = 0;
      l1 = p - 1;
    } else {              // S / N: along x1
      l0 = l1 = (s == 2) ? 0 : p - 1;
      k0 = 0;
      k1 = p - 1;
    }
    v += 0.5 * (opval(g, sD, sD2, sc, nbase, i, j, k0, l0) * g.E[q] +
                opval(g, sD, sD2, sc, nbase, i, j, k1, l1) * g.E[m + q]);
  }
  return v;
}

__device__ __forceinline__ void stage_tables(const Geom &g, double *sD, double *sD2) {
  const int pp = g.p * g.p;
  for (int e = threadIdx.x; e < pp; e += blockDim.x) {
    sD[e] = g.D[e];
    sD2[e] = g.D2[e];
  }
}

// Element (r, c) of the work matrix W = [A_ii | rhs] of one leaf (r, c
// counted in the padded layout), formed from the operator: used by the
// factorisation's first step, which builds W instead of reading it.
struct BuildSrc {
  int mode;           // RHS_CONDENSE or RHS_REFACTOR
  const double *f;    // [nleaf][ni] or nullptr (leaf-indexed like the geometry)
  const double *ub;   // [nleaf][nb] (RHS_REFACTOR)
};

__device__ __forceinline__ double build_elem(const Geom &g, LeafScale sc, int leaf,
                                             const BuildSrc &bs, int r, int c) {
  const int p = g.p, m = g.m, ni = g.ni, nb = g.nb, R = g.R;
  if (r >= ni) return (c == r) ? 1.0 : 0.0;
  const size_t nbase = (size_t)leaf * p * p;
  const int jr0 = (r * g.mdiv) >> 16;           // r / m (exact for r < 2048)
  const int i = r - jr0 * m + 1, j = jr0 + 1;
  if (c < ni) {
    const int lc0 = (c * g.mdiv) >> 16;
    const int k = c - lc0 * m + 1, l = lc0 + 1;
    if (!g.a12 && k != i && l != j) return 0.0;  // not on the row's grid lines
    return opval(g, g.D, g.D2, sc, nbase, i, j, k, l);
  }
  if (c < R) return 0.0;
  const int jr = c - R;
  if (bs.mode == RHS_CONDENSE) {
    if (jr < nb) return aib_elem(g, g.D, g.D2, sc, nbase, i, j, jr);
    if (jr == nb && bs.f) return bs.f[(size_t)leaf * ni + r];
    return 0.0;
  }
  if (jr != 0) return 0.0;
  const double *u = bs.ub + (size_t)leaf * nb;  // RHS_REFACTOR: f_i - A_ib u_b
  double v = bs.f ? bs.f[(size_t)leaf * ni + r] : 0.0;
  if (g.a12) {   // the mixed term couples the row to every slot
    for (int b = 0; b < nb; ++b) v -= aib_elem(g, g.D, g.D2, sc, nbase, i, j, b) * u[b];
    return v;
  }
  v -= opval(g, g.D, g.D2, sc, nbase, i, j, 0, j) * u[j - 1];
  v -= opval(g, g.D, g.D2, sc, nbase, i, j, p - 1, j) * u[m + j - 1];
  v -= opval(g, g.D, g.D2, sc, nbase, i, j, i, 0) * u[2 * m + i - 1];
  v -= opval(g, g.D, g.D2, sc, nbase, i, j, i, p - 1) * u[3 * m + i - 1];
  return v;
}

// Sparse formation of a 16-column tile of W = [A_ii | A_ib ...] (no mixed
// term): the column of node (k, l) is nonzero only in the rows of interior
// nodes on its two grid lines, (i, l) and (k, j), and a boundary node's
// column only on the one line that enters the leaf.  A tile qualifies when
// none of its columns is dense (the body-load or re-factor column).
__device__ __forceinline__ bool build_tile_sparse(const Geom &g, const BuildSrc &bs, int col0) {
  if (g.a12) return false;
  const int dense = bs.mode == RHS_CONDENSE ? (bs.f ? g.R + g.nb : -1) : g.R;
  return dense < col0 || dense >= col0 + 16;
}

// Entry q (0 <= q < 2m - 1) of column col's line list: the row node (i, j)
// and the column node (k, l); false when the column has no such entry (the
// right-hand-side columns hold A_ib only when condensing).
__device__ __forceinline__ bool line_entry(const Geom &g, const BuildSrc &bs, int col, int q,
                                           int &i, int &j, int &k, int &l) {
  const int m = g.m, p = g.p;
  if (col < g.ni) {
    k = col % m + 1;
    l = col / m + 1;
    if (q < m) {          // the x1-line through the node
      i = q + 1;
      j = l;
    } else {              // the x2-line, the node itself already counted
      i = k;
      j = q - m + 1;
      if (j >= l) ++j;
    }
    return true;
  }
  const int jr = col - g.R;
  if (bs.mode != RHS_CONDENSE || jr < 0 || jr >= g.nb || q >= m) return false;
  bnode(jr, m, p, k, l);
  if (k == 0 || k == p - 1) {   // W / E side: the x1-line of its row
    i = q + 1;
    j = l;
  } else {                      // S / N side: the x2-line of its column
    i = k;
    j = q + 1;
  }
  return true;
}

// Pivot search key of one candidate row: the magnitude's leading bits (exact
// for FP32; the top 32 bits of the FP64 pattern, i.e. 20 mantissa bits, so
// candidates within a relative 2^-20 of the largest count as ties) above the
// row index, complemented so that ties go to the lowest row.  Magnitudes of
// non-negative IEEE values order like their bit patterns; NaN sorts above
// infinity and is picked first, so it propagates.  0 marks "not a candidate".
__device__ __forceinline__ unsigned long long pivot_key(double v, int r) {
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(fabs(v)) >> 32);
  return ((unsigned long long)hi << 32) | (unsigned)(0x7fffffff - r);
}
__device__ __forceinline__ unsigned long long pivot_key(float v, int r) {
  const unsigned m = __float_as_uint(fabsf(v));
  return ((unsigned long long)m << 32) | (unsigned)(0x7fffffff - r);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_max_step(unsigned long long v) {
  const int lo = (int)(unsigned)v, hi = (int)(unsigned)(v >> 32);
  const int olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xf, false);
  const int ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xf, false);
  const unsigned long long o = ((unsigned long long)(unsigned)ohi << 32) | (unsigned)olo;
  return o > v ? o : v;
}

// Maximum of a 64-bit key over the wavefront with DPP moves (quad
// permutations, row shifts, then the row broadcasts of lanes 15 and 31);
// lane 63 ends with the maximum, which is read back to every lane.
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  v = dpp_max_step<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_max_step<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_max_step<0x114, 0xf>(v);  // row_shr:4
  v = dpp_max_step<0x118, 0xf>(v);  // row_shr:8
  v = dpp_max_step<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_max_step<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)v, 63);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
  return ((unsigned long long)hi << 32) | lo;
}

// One column C of the single-wavefront panel elimination.  The panel rows of
// a lane live in v[t][*] (row lane + 64t); C is a template argument so that
// every register index is static.
template <typename T, int C>
__device__ __forceinline__ void panel_column(T (&v)[4][16], unsigned &act, int lane, int R,
                                             int k, int *pv, int *rst, int *zeroPiv) {
  unsigned long long key = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if ((act >> t) & 1u) {
      const unsigned long long kt = pivot_key(v[t][C], lane + 64 * t);
      key = kt > key ? kt : key;
    }
  }
  key = wave_max_u64(key);
  int pr = 0x7fffffff - (int)(unsigned)(key & 0xffffffffu);
  pr = (pr >= 0 && pr < R) ? pr : R - 1;
  const int pt = pr >> 6, pl = pr & 63;
  if (lane == pl) act &= ~(1u << pt);
  // the pivot row (register pt of lane pl) is read into scalar registers;
  // every lane selects its register pt, lane pl's value is then broadcast
  // (no memory round trip, so no cross-lane ordering question)
  using B = typename std::conditional<sizeof(T) == 8, unsigned long long, unsigned>::type;
  const B m1 = (B)0 - (B)(pt & 1), m2 = (B)0 - (B)((pt >> 1) & 1);
  T pw[16];
#pragma unroll
  for (int cc = C; cc < 16; ++cc) {
    B b0, b1, b2, b3;
    __builtin_memcpy(&b0, &v[0][cc], sizeof(T));
    __builtin_memcpy(&b1, &v[1][cc], sizeof(T));
    __builtin_memcpy(&b2, &v[2][cc], sizeof(T));
    __builtin_memcpy(&b3, &v[3][cc], sizeof(T));
    const B b01 = (b0 & ~m1) | (b1 & m1), b23 = (b2 & ~m1) | (b3 & m1);
    const B bs = (b01 & ~m2) | (b23 & m2);
    B br;
    if constexpr (sizeof(T) == 8) {
      const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)bs, pl);
      const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(bs >> 32), pl);
      br = ((B)hi << 32) | lo;
    } else {
      br = (B)__builtin_amdgcn_readlane((int)bs, pl);
    }
    __builtin_memcpy(&pw[cc], &br, sizeof(T));
  }
  const T pval = pw[C];
  if (lane == 0) {
    pv[C] = pr;
    rst[pr] = k;
    if (pval == T(0) && *zeroPiv == 0) *zeroPiv = k * 16 + C + 1;
  }
  const T inv = (pval != T(0)) ? T(1) / pval : T(0);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if ((act >> t) & 1u) {
      const T l = v[t][C] * inv;
      v[t][C] = l;
#pragma unroll
      for (int cc = C + 1; cc < 16; ++cc) v[t][cc] -= l * pw[cc];
    }
  }
}

template <typename T, int... Cs>
__device__ __forceinline__ void panel_columns(T (&v)[4][16], unsigned &act, int lane, int R, int k,
                                              int *pv, int *rst, int *zeroPiv,
                                              std::integer_sequence<int, Cs...>) {
  (panel_column<T, Cs>(v, act, lane, R, k, pv, rst, zeroPiv), ...);
}

// ---------------------------------------------------------------------------
// factor: blocked LU with implicit partial pivoting, MFMA trailing updates
// ---------------------------------------------------------------------------
constexpr int kPST = 17;  // LDS row stride of the 16-column panel

template <typename T>
__device__ __forceinline__ T abs_key(T v) {
  T a = v < T(0) ? -v : v;
  return (a != a) ? T(INFINITY) : a;  // NaN is picked first, then propagates
}

// Workgroup-wide elimination of one 16-column panel held in LDS (R > 256),
// one barrier per column: after the barrier that publishes the wavefronts'
// candidates for column c, every thread picks the pivot (largest magnitude
// among the active rows, ties to the lowest row), updates its own rows'
// columns c ... 15, and right away scans its updated column c + 1 for the
// next pivot candidate; one barrier then publishes both the updated rows
// and the new candidates (kept in two slots by column parity, so that a
// slot is not rewritten while it may still be read).  The pivot row is not
// touched by the update, so every thread may read it while others update.
template <typename T, int NT>
__device__ __forceinline__ void panel_wg(T *P, int R, int k, int *pv, int *rst, int *zeroPiv,
                                         T *redv, int *redi) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  auto publish = [&](T best, int bi, int slot) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const T ob = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) { redv[slot * NW + wv] = best; redi[slot * NW + wv] = bi; }
  };
  {
    T best = T(-1);
    int bi = INT_MAX;
    for (int r = tid; r < R; r += NT) {
      if (rst[r] != kInfoActive) continue;
      const T v = abs_key(P[r * kPST]);
      if (v > best) { best = v; bi = r; }
    }
    publish(best, bi, 0);
  }
  __syncthreads();
  for (int c = 0; c < 16; ++c) {
    const int slot = c & 1;
    T best = redv[slot * NW];
    int bi = redi[slot * NW];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      const T ob = redv[slot * NW + w];
      const int oi = redi[slot * NW + w];
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    // R - (16k + c) >= 1 rows are active, so bi is a valid row; the clamp
    // only guards the memory access.
    const int pr = bi < R ? bi : R - 1;
    const T pval = P[pr * kPST + c];
    if (tid == 0) {
      pv[c] = pr;
      rst[pr] = k;
      if (pval == T(0) && *zeroPiv == 0) *zeroPiv = k * 16 + c + 1;
    }
    const T inv = (pval != T(0)) ? T(1) / pval : T(0);
    T nbest = T(-1);
    int nbi = INT_MAX;
    for (int r = tid; r < R; r += NT) {
      if (r == pr || rst[r] != kInfoActive) continue;
      const T l = P[r * kPST + c] * inv;
      P[r * kPST + c] = l;
      for (int cc = c + 1; cc < 16; ++cc) P[r * kPST + cc] -= l * P[pr * kPST + cc];
      if (c + 1 < 16) {
        const T v = abs_key(P[r * kPST + c + 1]);
        if (v > nbest) { nbest = v; nbi = r; }
      }
    }
    if (c + 1 < 16) publish(nbest, nbi, slot ^ 1);
    __syncthreads();
  }
}

template <typename T, int NT>
__global__ void __launch_bounds__(NT, 512 / NT) k_factor(Geom g, T *M, int *piv, int *rstep,
                                                        int *info, int CH, Sel sel, BuildSrc bs) {
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  const int wi = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int leaf;
  if (!resolve_leaf(sel, leaf)) return;
  const int R = g.R, RT = g.RT, CT = g.CT;
  const int UST = CH + 16;
  T *P = (T *)smem;                       // [R][kPST]   panel
  T *U = P + (size_t)R * kPST;            // [16][UST]   U12 chunk
  T *Linv = U + 16 * UST;                 // [16][kPST]  inverse of L11
  T *redv = Linv + 16 * kPST;             // [2][NW]
  int *rst = (int *)(redv + 2 * NW);      // [R]         retire step
  int *tileAct = rst + R;                 // [RT]
  int *pv = tileAct + RT;                 // [16]
  int *redi = pv + 16;                    // [2][NW]
  int *zeroPiv = redi + 2 * NW;           // [1]
  T *Ml = M + leaf_stride(g) * wi;
  const LeafScale sc = leaf_scale(g, leaf);

  for (int r = tid; r < R; r += NT) rst[r] = kInfoActive;
  if (tid == 0) *zeroPiv = 0;
  // form W from the operator (coalesced, tile-major); the leaf's matrix is
  // read back by this workgroup right away, mostly from cache
  {
    const size_t total = work_elems(g);
    for (size_t e = tid; e < total; e += NT) {
      const int tile = (int)(e >> 8);
      int ri, ci;
      Tile<T>::rc((int)(e & 255), ri, ci);
      Ml[e] = (T)build_elem(g, sc, leaf, bs, (tile / CT) * 16 + ri, (tile % CT) * 16 + ci);
    }
  }
  __syncthreads();

  for (int k = 0; k < RT; ++k) {
    for (int e = tid; e < R * 16; e += NT) {
      const int r = e >> 4, c = e & 15;
      P[r * kPST + c] = Ml[tix<T>(r, k * 16 + c, CT)];
    }
    __syncthreads();

    // --- panel: 16 columns of unblocked elimination in LDS ---
    if constexpr (NT == 256) {
      // One wavefront: lane l owns rows l, l+64, l+128, l+192 and keeps
      // their active bits in a register, so no workgroup barrier is needed
      // between columns (LDS accesses of one wave are ordered).
      if (wv == 0) {
        // one wavefront, the panel in registers: lane l owns rows
        // l + 64t (t < 4); the pivot search is a DPP maximum of pivot_key.
        T v[4][16];
        unsigned act = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int r = lane + 64 * t;
          const bool in = r < R;
          if (in && rst[r] == kInfoActive) act |= 1u << t;
#pragma unroll
          for (int c = 0; c < 16; ++c) v[t][c] = in ? P[r * kPST + c] : T(0);
        }
        panel_columns<T>(v, act, lane, R, k, pv, rst, zeroPiv,
                         std::make_integer_sequence<int, 16>());
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int r = lane + 64 * t;
          if (r < R) {
#pragma unroll
            for (int c = 0; c < 16; ++c) P[r * kPST + c] = v[t][c];
          }
        }
      }
      __syncthreads();
    } else {
      panel_wg<T, NT>(P, R, k, pv, rst, zeroPiv, redv, redi);
    }

    // L11^{-1} (unit lower triangular, rows in pivot order): column j of the
    // inverse by forward substitution in lane j of wave 0
    if (wv == 0 && lane < 16) {
      const int j = lane;
      T x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        T acc = (i == j) ? T(1) : T(0);
#pragma unroll
        for (int q = 0; q < i; ++q) acc -= P[pv[i] * kPST + q] * x[q];
        x[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) Linv[i * kPST + j] = x[i];
    }
    for (int t = tid; t < RT; t += NT) {
      int a = 0;
      for (int q = 0; q < 16; ++q) a |= (rst[t * 16 + q] == kInfoActive);
      tileAct[t] = a;
    }
    __syncthreads();

    // --- U12 = L11^{-1} A12 and the trailing update, in column chunks ---
    const int cend = CT * 16;
    for (int c0 = (k + 1) * 16; c0 < cend; c0 += CH) {
      const int cw = min(CH, cend - c0);
      // gather the raw pivot rows of the chunk (16 contiguous elements of a
      // row per tile)
      for (int e = tid; e < 16 * cw; e += NT) {
        const int sr = e / cw, cc = e - sr * cw;
        U[sr * UST + cc] = Ml[tix<T>(pv[sr], c0 + cc, CT)];
      }
      __syncthreads();
      // U12 = L11^{-1} A12 on MFMA, one tile per wave at a time, in place in
      // U; the pivot rows of W receive their U12 entries
      for (int jl = wv; jl < (cw >> 4); jl += NW) {
        typename Mfma<T>::acc acc;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = T(0);
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
          const T a = Linv[(lane & 15) * kPST + 4 * kc + (lane >> 4)];
          const T b = U[(4 * kc + (lane >> 4)) * UST + jl * 16 + (lane & 15)];
          acc = Mfma<T>::op(a, b, acc);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int sr = Tile<T>::crow(q, lane);
          const int cc = jl * 16 + (lane & 15);
          U[sr * UST + cc] = acc[q];
          Ml[tix<T>(pv[sr], c0 + cc, CT)] = acc[q];
        }
      }
      __syncthreads();
      // strips of up to four column tiles of one row tile per wave: all
      // loads of a strip are in flight together and the A operand is shared
      const int ntj = cw >> 4;
      const int nstrip = (ntj + 3) >> 2;
      for (int t = wv; t < RT * nstrip; t += NW) {
        const int ti = t / nstrip, j0 = (t - ti * nstrip) * 4;
        if (!tileAct[ti]) continue;
        const int nj = min(4, ntj - j0);
        T *Ct = Ml + ((size_t)(ti * CT + (c0 >> 4) + j0) << 8);
        typename Mfma<T>::acc acc[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          if (jj < nj) {
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[jj][q] = Ct[jj * 256 + q * 64 + lane];
          }
        }
        const int ar = ti * 16 + (lane & 15);
        const bool act = rst[ar] == kInfoActive;
        T a[4];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) a[kc] = act ? -P[ar * kPST + 4 * kc + (lane >> 4)] : T(0);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          if (jj < nj) {
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
              const T b = U[(4 * kc + (lane >> 4)) * UST + (j0 + jj) * 16 + (lane & 15)];
              acc[jj] = Mfma<T>::op(a[kc], b, acc[jj]);
            }
          }
        }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          if (jj < nj) {
#pragma unroll
            for (int q = 0; q < 4; ++q) Ct[jj * 256 + q * 64 + lane] = acc[jj][q];
          }
        }
      }
      __syncthreads();
    }

    for (int e = tid; e < R * 16; e += NT) {
      const int r = e >> 4, c = e & 15;
      Ml[tix<T>(r, k * 16 + c, CT)] = P[r * kPST + c];
    }
    if (tid < 16) piv[(size_t)wi * R + k * 16 + tid] = pv[tid];
    __syncthreads();
  }
  for (int r = tid; r < R; r += NT) rstep[(size_t)wi * R + r] = rst[r];
  if (tid == 0) info[leaf] = *zeroPiv;
}

// ---------------------------------------------------------------------------
// factor2: the same factorisation for R <= 256 with panels taken in pairs.
// Panel A's update is applied at once only to panel B's column tile; panel
// B is factored, and the rest of the trailing matrix then receives both
// updates in one pass (C -= L21_A U12_A + L21_B U12_B, 8 MFMAs per tile), so
// the trailing matrix streams through memory half as often.  The pivot rows
// of B take panel A's update on the way: U12_B = L11_B^{-1} (A12_B -
// L21_A[B] U12_A).  The stored form (multipliers in the panel columns, U rows
// in the pivot rows, retire steps) is exactly that of k_factor.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void panel_one_wave(T *P, int R, int k, int lane, int *pv, int *rst,
                                               int *zeroPiv) {
  T v[4][16];
  unsigned act = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = lane + 64 * t;
    const bool in = r < R;
    if (in && rst[r] == kInfoActive) act |= 1u << t;
#pragma unroll
    for (int c = 0; c < 16; ++c) v[t][c] = in ? P[r * kPST + c] : T(0);
  }
  panel_columns<T>(v, act, lane, R, k, pv, rst, zeroPiv, std::make_integer_sequence<int, 16>());
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = lane + 64 * t;
    if (r < R) {
#pragma unroll
      for (int c = 0; c < 16; ++c) P[r * kPST + c] = v[t][c];
    }
  }
}

// L11^{-1} of a factored panel (unit lower triangular, rows in pivot order);
// lane j < 16 forms column j by forward substitution.
template <typename T>
__device__ __forceinline__ void linv16(const T *P, const int *pv, T *Linv, int lane) {
  if (lane < 16) {
    const int j = lane;
    T x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      T acc = (i == j) ? T(1) : T(0);
#pragma unroll
      for (int q = 0; q < i; ++q) acc -= P[pv[i] * kPST + q] * x[q];
      x[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) Linv[i * kPST + j] = x[i];
  }
}

// D (16x16 tile, accumulator layout) = L (16x16, LDS row-major stride kPST)
// times the tile of B at column offset bc in a row-major LDS block.
template <typename T>
__device__ __forceinline__ typename Mfma<T>::acc tri_apply(const T *L, const T *B, int BST, int bc,
                                                           int lane) {
  typename Mfma<T>::acc acc;
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = T(0);
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    const T a = L[(lane & 15) * kPST + 4 * kc + (lane >> 4)];
    const T b = B[(4 * kc + (lane >> 4)) * BST + bc + (lane & 15)];
    acc = Mfma<T>::op(a, b, acc);
  }
  return acc;
}

template <typename T>
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename T, int MINB>
__global__ void __launch_bounds__(256, MINB) k_factor2_t(Geom g, T *M, int *piv, int *rstep,
                                                    int *info, int CH, Sel sel, BuildSrc bs) {
  constexpr int NT = 256, NW = 4;
  extern __shared__ __align__(16) unsigned char smem[];
  const int wi = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int leaf;
  if (!resolve_leaf(sel, leaf)) return;
  const int R = g.R, RT = g.RT, CT = g.CT;
  const int UST = CH + 16;
  T *PA = (T *)smem;                      // [R][kPST]  panel A
  T *PB = PA + (size_t)R * kPST;          // [R][kPST]  panel B
  T *U = PB + (size_t)R * kPST;           // [32][UST]  raw / U12 rows of A (0..15), B (16..31)
  T *LA = U + 32 * UST;                   // [16][kPST] L11_A^{-1}
  T *LB = LA + 16 * kPST;                 // [16][kPST] L11_B^{-1}
  int *rst = (int *)(LB + 16 * kPST);     // [R]
  int *tileAct = rst + R;                 // [RT]
  int *pvA = tileAct + RT;                // [16]
  int *pvB = pvA + 16;                    // [16]
  int *zeroPiv = pvB + 16;                // [1]
  T *Ml = M + leaf_stride(g) * wi;
  const LeafScale sc = leaf_scale(g, leaf);

  for (int r = tid; r < R; r += NT) rst[r] = kInfoActive;
  if (tid == 0) *zeroPiv = 0;
  {
    const size_t total = work_elems(g);
    for (size_t e = tid; e < total; e += NT) {
      const int tile = (int)(e >> 8);
      int ri, ci;
      Tile<T>::rc((int)(e & 255), ri, ci);
      Ml[e] = (T)build_elem(g, sc, leaf, bs, (tile / CT) * 16 + ri, (tile % CT) * 16 + ci);
    }
  }
  __syncthreads();

  auto load_panel = [&](T *Pb, int k) {
    for (int e = tid; e < R * 16; e += NT) {
      const int r = e >> 4, c = e & 15;
      Pb[r * kPST + c] = Ml[tix<T>(r, k * 16 + c, CT)];
    }
  };
  auto factor_panel = [&](T *Pb, int k, int *pv, T *Li) {
    if (wv == 0) {
      panel_one_wave<T>(Pb, R, k, lane, pv, rst, zeroPiv);
      // pv and rst were written by lane 0 alone: order those writes before
      // the other lanes read them
      wave_lds_fence<T>();
      linv16<T>(Pb, pv, Li, lane);
      for (int t = lane; t < RT; t += 64) {
        int a = 0;
        for (int q = 0; q < 16; ++q) a |= (rst[t * 16 + q] == kInfoActive);
        tileAct[t] = a;
      }
    }
  };
  // C -= sum over the panels in use of L21 U12, strips of up to 4 tiles of
  // one row tile per wave; the next strip's tiles are loaded before the
  // current strip's MFMAs so that two strips per wave are in flight.
  auto trailing = [&](int c0, int cw, bool two) {
    const int ntj = cw >> 4;
    const int nstrip = (ntj + 3) >> 2;
    const int nall = RT * nstrip;
    auto next_strip = [&](int t) {
      while (t < nall && !tileAct[t / nstrip]) t += NW;
      return t;
    };
    typename Mfma<T>::acc cur[4], nxt[4];
    auto load_strip = [&](int t, typename Mfma<T>::acc (&dst)[4]) {
      const int ti = t / nstrip, j0 = (t - ti * nstrip) * 4;
      const int nj = min(4, ntj - j0);
      const T *Ct = Ml + ((size_t)(ti * CT + (c0 >> 4) + j0) << 8);
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        if (jj < nj) {
#pragma unroll
          for (int q = 0; q < 4; ++q) dst[jj][q] = Ct[jj * 256 + q * 64 + lane];
        }
      }
    };
    int t = next_strip(wv);
    if (t < nall) load_strip(t, cur);
    while (t < nall) {
      const int tn = next_strip(t + NW);
      if (tn < nall) load_strip(tn, nxt);
      const int ti = t / nstrip, j0 = (t - ti * nstrip) * 4;
      const int nj = min(4, ntj - j0);
      const int ar = ti * 16 + (lane & 15);
      const bool act = rst[ar] == kInfoActive;
      T a[8];
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        a[kc] = act ? -PA[ar * kPST + 4 * kc + (lane >> 4)] : T(0);
        a[4 + kc] = (act && two) ? -PB[ar * kPST + 4 * kc + (lane >> 4)] : T(0);
      }
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        if (jj < nj) {
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) {
            const T b = U[(4 * kc + (lane >> 4)) * UST + (j0 + jj) * 16 + (lane & 15)];
            cur[jj] = Mfma<T>::op(a[kc], b, cur[jj]);
          }
          if (two) {
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
              const T b = U[(16 + 4 * kc + (lane >> 4)) * UST + (j0 + jj) * 16 + (lane & 15)];
              cur[jj] = Mfma<T>::op(a[4 + kc], b, cur[jj]);
            }
          }
        }
      }
      T *Ct = Ml + ((size_t)(ti * CT + (c0 >> 4) + j0) << 8);
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        if (jj < nj) {
#pragma unroll
          for (int q = 0; q < 4; ++q) Ct[jj * 256 + q * 64 + lane] = cur[jj][q];
        }
      }
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) cur[jj] = nxt[jj];
      t = tn;
    }
  };
  // Pivot rows of A (and B) over columns [c0, c0+cw): U12 rows, stored in W.
  auto u12 = [&](int c0, int cw, bool two) {
    const int nrow = two ? 32 : 16;
    for (int e = tid; e < nrow * cw; e += NT) {
      const int sr = e / cw, cc = e - sr * cw;
      const int row = sr < 16 ? pvA[sr] : pvB[sr - 16];
      U[sr * UST + cc] = Ml[tix<T>(row, c0 + cc, CT)];
    }
    __syncthreads();
    for (int jl = wv; jl < (cw >> 4); jl += NW) {
      const int cb = jl * 16 + (lane & 15);
      typename Mfma<T>::acc ua = tri_apply<T>(LA, U, UST, jl * 16, lane);
      wave_lds_fence<T>();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int sr = Tile<T>::crow(q, lane);
        U[sr * UST + cb] = ua[q];
        Ml[tix<T>(pvA[sr], c0 + cb, CT)] = ua[q];
      }
      if (two) {
        wave_lds_fence<T>();
        // raw rows of B minus panel A's update: U_B - L21_A[pvB] U12_A
        typename Mfma<T>::acc ub;
#pragma unroll
        for (int q = 0; q < 4; ++q) ub[q] = U[(16 + Tile<T>::crow(q, lane)) * UST + cb];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
          const T a = -PA[pvB[lane & 15] * kPST + 4 * kc + (lane >> 4)];
          const T b = U[(4 * kc + (lane >> 4)) * UST + cb];
          ub = Mfma<T>::op(a, b, ub);
        }
        wave_lds_fence<T>();
#pragma unroll
        for (int q = 0; q < 4; ++q) U[(16 + Tile<T>::crow(q, lane)) * UST + cb] = ub[q];
        wave_lds_fence<T>();
        typename Mfma<T>::acc u2 = tri_apply<T>(LB, U + 16 * UST, UST, jl * 16, lane);
        wave_lds_fence<T>();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int sr = Tile<T>::crow(q, lane);
          U[(16 + sr) * UST + cb] = u2[q];
          Ml[tix<T>(pvB[sr], c0 + cb, CT)] = u2[q];
        }
      }
    }
    __syncthreads();
  };

  for (int k = 0; k < RT; k += 2) {
    const bool two = k + 1 < RT;
    load_panel(PA, k);
    __syncthreads();
    factor_panel(PA, k, pvA, LA);
    __syncthreads();
    if (two) {
      // panel A's update of panel B's column tile only
      u12(16 * (k + 1), 16, false);
      trailing(16 * (k + 1), 16, false);
      __syncthreads();
      load_panel(PB, k + 1);
      __syncthreads();
      factor_panel(PB, k + 1, pvB, LB);
      __syncthreads();
    }
    const int cend = CT * 16;
    for (int c0 = 16 * (k + (two ? 2 : 1)); c0 < cend; c0 += CH) {
      const int cw = min(CH, cend - c0);
      u12(c0, cw, two);
      trailing(c0, cw, two);
      __syncthreads();
    }
    for (int e = tid; e < R * 16; e += NT) {
      const int r = e >> 4, c = e & 15;
      Ml[tix<T>(r, k * 16 + c, CT)] = PA[r * kPST + c];
      if (two) Ml[tix<T>(r, (k + 1) * 16 + c, CT)] = PB[r * kPST + c];
    }
    if (tid < 16) piv[(size_t)wi * R + k * 16 + tid] = pvA[tid];
    if (two && tid >= 16 && tid < 32) piv[(size_t)wi * R + (k + 1) * 16 + tid - 16] = pvB[tid - 16];
    __syncthreads();
  }
  for (int r = tid; r < R; r += NT) rstep[(size_t)wi * R + r] = rst[r];
  if (tid == 0) info[leaf] = *zeroPiv;
}

// ---------------------------------------------------------------------------
// factorP: panels in pairs for R > 256 (up to p = 32), where two panels do
// not fit LDS together.  Panel A is factored in the LDS panel buffer and
// written back to the work matrix; A's update reaches panel B's column tile;
// panel B is loaded into the same buffer and factored; the remaining columns
// then take both updates in one pass, C -= L21_A U12_A + L21_B U12_B, with
// L21_A read back from the work matrix (where it was just written, so
// mostly from L2) and L21_B from LDS.  The trailing matrix thus streams
// through HBM once per 32 columns instead of once per 16.  The stored form
// is that of k_factor.
// ---------------------------------------------------------------------------
template <typename T, int NT, int MINW>
__global__ void __launch_bounds__(NT, MINW) k_factorP(Geom g, T *M, int *piv, int *rstep,
                                                     int *info, int CH, Sel sel, BuildSrc bs) {
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  const int wi = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int leaf;
  if (!resolve_leaf(sel, leaf)) return;
  const int R = g.R, RT = g.RT, CT = g.CT;
  const int UST = CH + 16;
  T *P = (T *)smem;                       // [R][kPST]   current panel
  T *U = P + (size_t)R * kPST;            // [32][UST]   U12 rows of A (0..15), B (16..31)
  T *LA = U + 32 * UST;                   // [16][kPST]  L11_A^{-1}
  T *LB = LA + 16 * kPST;                 // [16][kPST]  L11_B^{-1}
  T *redv = LB + 16 * kPST;               // [2][NW]
  int *rst = (int *)(redv + 2 * NW);      // [R]
  int *tileAct = rst + R;                 // [RT]
  int *pvA = tileAct + RT;                // [16]
  int *pvB = pvA + 16;                    // [16]
  int *redi = pvB + 16;                   // [2][NW]
  int *zeroPiv = redi + 2 * NW;           // [1]
  T *Ml = M + leaf_stride(g) * wi;
  const LeafScale sc = leaf_scale(g, leaf);

  for (int r = tid; r < R; r += NT) rst[r] = kInfoActive;
  if (tid == 0) *zeroPiv = 0;
  {
    const size_t total = work_elems(g);
    for (size_t e = tid; e < total; e += NT) {
      const int tile = (int)(e >> 8);
      int ri, ci;
      Tile<T>::rc((int)(e & 255), ri, ci);
      Ml[e] = (T)build_elem(g, sc, leaf, bs, (tile / CT) * 16 + ri, (tile % CT) * 16 + ci);
    }
  }
  __syncthreads();

  // factor the panel of column tile kk into P, L11^{-1} into Li, pivots into
  // pv and the global pivot list, active row-tile flags; the factored panel
  // is also written back to the work matrix
  auto do_panel = [&](int kk, int *pv, T *Li) {
    for (int e = tid; e < R * 16; e += NT) {
      const int r = e >> 4, c = e & 15;
      P[r * kPST + c] = Ml[tix<T>(r, kk * 16 + c, CT)];
    }
    __syncthreads();
    panel_wg<T, NT>(P, R, kk, pv, rst, zeroPiv, redv, redi);
    if (wv == 0 && lane < 16) {
      const int j = lane;
      T x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        T acc = (i == j) ? T(1) : T(0);
#pragma unroll
        for (int q = 0; q < i; ++q) acc -= P[pv[i] * kPST + q] * x[q];
        x[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) Li[i * kPST + j] = x[i];
      piv[(size_t)wi * R + kk * 16 + j] = pv[j];
    }
    for (int t = tid; t < RT; t += NT) {
      int a = 0;
      for (int q = 0; q < 16; ++q) a |= (rst[t * 16 + q] == kInfoActive);
      tileAct[t] = a;
    }
    for (int e = tid; e < R * 16; e += NT) {
      const int r = e >> 4, c = e & 15;
      Ml[tix<T>(r, kk * 16 + c, CT)] = P[r * kPST + c];
    }
    __syncthreads();
  };
  // U12 rows over columns [c0, c0+cw): A's from its raw pivot rows, B's
  // (two) from its raw pivot rows minus A's update at them; both written to
  // U and into the pivot rows of W
  auto u12 = [&](int k, int c0, int cw, bool two) {
    const int nrow = two ? 32 : 16;
    for (int e = tid; e < nrow * cw; e += NT) {
      const int sr = e / cw, cc = e - sr * cw;
      const int row = sr < 16 ? pvA[sr] : pvB[sr - 16];
      U[sr * UST + cc] = Ml[tix<T>(row, c0 + cc, CT)];
    }
    __syncthreads();
    for (int jl = wv; jl < (cw >> 4); jl += NW) {
      const int cb = jl * 16 + (lane & 15);
      typename Mfma<T>::acc ua = tri_apply<T>(LA, U, UST, jl * 16, lane);
      wave_lds_fence<T>();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int sr = Tile<T>::crow(q, lane);
        U[sr * UST + cb] = ua[q];
        Ml[tix<T>(pvA[sr], c0 + cb, CT)] = ua[q];
      }
      if (two) {
        wave_lds_fence<T>();
        typename Mfma<T>::acc ub;
#pragma unroll
        for (int q = 0; q < 4; ++q) ub[q] = U[(16 + Tile<T>::crow(q, lane)) * UST + cb];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
          const T a = -Ml[tix<T>(pvB[lane & 15], k * 16 + 4 * kc + (lane >> 4), CT)];
          const T b = U[(4 * kc + (lane >> 4)) * UST + cb];
          ub = Mfma<T>::op(a, b, ub);
        }
        wave_lds_fence<T>();
#pragma unroll
        for (int q = 0; q < 4; ++q) U[(16 + Tile<T>::crow(q, lane)) * UST + cb] = ub[q];
        wave_lds_fence<T>();
        typename Mfma<T>::acc u2 = tri_apply<T>(LB, U + 16 * UST, UST, jl * 16, lane);
        wave_lds_fence<T>();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int sr = Tile<T>::crow(q, lane);
          U[(16 + sr) * UST + cb] = u2[q];
          Ml[tix<T>(pvB[sr], c0 + cb, CT)] = u2[q];
        }
      }
    }
    __syncthreads();
  };
  // C -= L21_A U12_A (+ L21_B U12_B) on the active row tiles over columns
  // [c0, c0+cw); L21_A from the work matrix when two, else from P
  auto trailing = [&](int k, int c0, int cw, bool two) {
    const int ntj = cw >> 4;
    const int nstrip = (ntj + 3) >> 2;
    for (int t = wv; t < RT * nstrip; t += NW) {
      const int ti = t / nstrip, j0 = (t - ti * nstrip) * 4;
      if (!tileAct[ti]) continue;
      const int nj = min(4, ntj - j0);
      T *Ct = Ml + ((size_t)(ti * CT + (c0 >> 4) + j0) << 8);
      typename Mfma<T>::acc acc[4];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        if (jj < nj) {
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[jj][q] = Ct[jj * 256 + q * 64 + lane];
        }
      }
      const int ar = ti * 16 + (lane & 15);
      const bool act = rst[ar] == kInfoActive;
      // one 16-deep update at a time: L21 from the work matrix (panel A of
      // a pair) or from P (the last panel taken)
      for (int h = two ? 0 : 1; h < 2; ++h) {
        T a[4];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
          const int ac = 4 * kc + (lane >> 4);
          a[kc] = act ? -(h == 0 ? Ml[tix<T>(ar, k * 16 + ac, CT)] : P[ar * kPST + ac]) : T(0);
        }
        const T *Uh = U + (two && h == 1 ? 16 * UST : 0);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          if (jj < nj) {
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
              const T b = Uh[(4 * kc + (lane >> 4)) * UST + (j0 + jj) * 16 + (lane & 15)];
              acc[jj] = Mfma<T>::op(a[kc], b, acc[jj]);
            }
          }
        }
      }
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        if (jj < nj) {
#pragma unroll
          for (int q = 0; q < 4; ++q) Ct[jj * 256 + q * 64 + lane] = acc[jj][q];
        }
      }
    }
    __syncthreads();
  };

  const int cend = CT * 16;
  for (int k = 0; k < RT; k += 2) {
    const bool two = k + 1 < RT;
    do_panel(k, pvA, LA);
    if (two) {
      // panel A's update of panel B's column tile (P still holds panel A)
      u12(k, 16 * (k + 1), 16, false);
      trailing(k, 16 * (k + 1), 16, false);
      do_panel(k + 1, pvB, LB);
    }
    for (int c0 = 16 * (k + (two ? 2 : 1)); c0 < cend; c0 += CH) {
      const int cw = min(CH, cend - c0);
      u12(k, c0, cw, two);
      trailing(k, c0, cw, two);
    }
  }
  for (int r = tid; r < R; r += NT) rstep[(size_t)wi * R + r] = rst[r];
  if (tid == 0) info[leaf] = *zeroPiv;
}

// ---------------------------------------------------------------------------
// Operator tables staged in LDS for one leaf: D, D^2 (p x p) and the
// coefficient samples of the leaf (p x p each, absent ones NULL), so that
// forming W reads no global memory per element.
// ---------------------------------------------------------------------------
struct StagedOp {
  const double *D, *D2, *a11, *c1, *a22, *c2, *k2b;
};

__device__ __forceinline__ double opval_s(int p, const StagedOp &t, LeafScale sc, int i, int j,
                                          int k, int l) {
  const int n = i + p * j;
  double v = 0.0;
  if (l == j) {
    const double a = t.a11 ? t.a11[n] : 1.0;
    const double c = t.c1 ? t.c1[n] : 0.0;
    v -= a * (sc.sx * sc.sx) * t.D2[i * p + k] + c * sc.sx * t.D[i * p + k];
  }
  if (k == i) {
    const double a = t.a22 ? t.a22[n] : 1.0;
    const double c = t.c2 ? t.c2[n] : 0.0;
    v -= a * (sc.sy * sc.sy) * t.D2[j * p + l] + c * sc.sy * t.D[j * p + l];
  }
  if (k == i && l == j && t.k2b) v -= t.k2b[n];
  return v;
}

// build_elem with the tables in LDS (condensation right-hand sides only)
__device__ __forceinline__ double build_elem_s(const Geom &g, const StagedOp &t, LeafScale sc,
                                               int leaf, const double *f, int r, int c) {
  const int p = g.p, m = g.m, ni = g.ni, nb = g.nb, R = g.R;
  if (r >= ni) return (c == r) ? 1.0 : 0.0;
  const int i = r % m + 1, j = r / m + 1;
  if (c < ni) return opval_s(p, t, sc, i, j, c % m + 1, c / m + 1);
  if (c < R) return 0.0;
  const int jr = c - R;
  if (jr < nb) {
    int k, l;
    bnode(jr, m, p, k, l);
    return opval_s(p, t, sc, i, j, k, l);
  }
  if (jr == nb && f) return f[(size_t)leaf * ni + r];
  return 0.0;
}

// Wavefront maximum of a 32-bit key (DPP as in wave_max_u64); every lane
// receives it.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xb1, 0xf, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4e, 0xf, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x114, 0xf, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x118, 0xf, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xa, 0xf, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xc, 0xf, false));
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// One column C of the FP32 single-wavefront panel of factor_rr.  Rows of a
// lane: v[t][*] = row lane + 64t (R <= 256).  The pivot rule is that of
// panel_column up to the key's resolution (the top 24 bits of the FP32
// magnitude above the complemented row index: candidates within a relative
// 2^-16 count as ties, the lowest row wins).  The pivot row is broadcast
// through LDS and the multipliers use the reciprocal of the pivot.
template <int C>
__device__ __forceinline__ void rr_panel_column(float (&v)[4][16], unsigned &act, int lane, int k,
                                                float *prb, int *pv, int *rst, int &zp) {
  unsigned key = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if ((act >> t) & 1u) {
      const unsigned kt = ((__float_as_uint(fabsf(v[t][C])) >> 7) << 8) | (unsigned)(255 - (lane + 64 * t));
      key = max(key, kt);
    }
  }
  key = wave_max_u32(key);
  const int pr = 255 - (int)(key & 255u);
  const int pt = pr >> 6, pl = pr & 63;
  if (lane == pl) {
    act &= ~(1u << pt);
    // register pt selected by bit masks (a select of values, which the
    // compiler would otherwise turn into an indexed, memory-backed access)
    const unsigned m1 = 0u - (unsigned)(pt & 1), m2 = 0u - (unsigned)((pt >> 1) & 1);
#pragma unroll
    for (int cc = C; cc < 16; ++cc) {
      const unsigned b0 = __float_as_uint(v[0][cc]), b1 = __float_as_uint(v[1][cc]);
      const unsigned b2 = __float_as_uint(v[2][cc]), b3 = __float_as_uint(v[3][cc]);
      const unsigned b01 = (b0 & ~m1) | (b1 & m1), b23 = (b2 & ~m1) | (b3 & m1);
      prb[cc] = __uint_as_float((b01 & ~m2) | (b23 & m2));
    }
  }
  wave_lds_fence<float>();
  float pw[16];
#pragma unroll
  for (int cc = C; cc < 16; ++cc) pw[cc] = prb[cc];
  const float pval = pw[C];
  if (lane == 0) {
    pv[C] = pr;
    rst[pr] = k;
    if (pval == 0.0f && zp == 0) zp = k * 16 + C + 1;
  }
  const float inv = pval != 0.0f ? __builtin_amdgcn_rcpf(pval) : 0.0f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if ((act >> t) & 1u) {
      const float l = v[t][C] * inv;
      v[t][C] = l;
#pragma unroll
      for (int cc = C + 1; cc < 16; ++cc) v[t][cc] = fmaf(-l, pw[cc], v[t][cc]);
    }
  }
  wave_lds_fence<float>();
}

template <int... Cs>
__device__ __forceinline__ void rr_panel_columns(float (&v)[4][16], unsigned &act, int lane, int k,
                                                 float *prb, int *pv, int *rst, int &zp,
                                                 std::integer_sequence<int, Cs...>) {
  (rr_panel_column<Cs>(v, act, lane, k, prb, pv, rst, zp), ...);
}

// panel_wg with the panel rows in registers: thread t holds panel rows t,
// t + NT, ... (all 16 columns), so each column's update is register
// arithmetic instead of LDS traffic.  Before each barrier every wavefront
// publishes its candidate for the coming column, a DPP maximum of the
// packed pivot key (magnitude's leading bits, then the complemented row:
// ties to the lowest row, as in the single-wavefront panel), with the
// candidate row's values, stored by the lane that holds the row; after it
// every thread takes the largest of the wavefronts' keys, updates its rows
// and scans the next column.  Slots alternate by column parity.  The rows
// go back to LDS at the end, where the rest of the factorisation reads them.
struct PanelSlots {
  unsigned long long *key;   // [2][NW] the wavefronts' candidate keys (0: none)
  void *vals;                // [2][NW][16] the candidate rows' values
};

template <typename T, int NT, int RPT, int C>
__device__ __forceinline__ void preg_publish(const T (&v)[RPT][16], const bool (&act)[RPT],
                                             int tid, const PanelSlots &ps) {
  constexpr int NW = NT / 64;
  const int lane = tid & 63, wv = tid >> 6, slot = (C & 1) * NW + wv;
  unsigned long long key = 0;
#pragma unroll
  for (int h = 0; h < RPT; ++h) {
    if (act[h]) {
      const unsigned long long kh = pivot_key(v[h][C], tid + h * NT);
      key = kh > key ? kh : key;
    }
  }
  const unsigned long long wk = wave_max_u64(key);
  const int wr = 0x7fffffff - (int)(unsigned)(wk & 0xffffffffu);   // INT_MAX: no active row
  T *dst = (T *)ps.vals + slot * 16;
  if (lane == 0) ps.key[slot] = wk;
  if (wk == 0 && lane < 16) dst[lane] = T(0);
#pragma unroll
  for (int h = 0; h < RPT; ++h) {
    if (tid + h * NT == wr) {
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) dst[cc] = v[h][cc];
    }
  }
}

template <typename T, int NT, int RPT, int C>
__device__ __forceinline__ void preg_column(T (&v)[RPT][16], bool (&act)[RPT], int tid, int R,
                                            int k, int *pv, int *rst, int *zeroPiv,
                                            const PanelSlots &ps) {
  constexpr int NW = NT / 64;
  const int s0 = (C & 1) * NW;
  const T *vals = (const T *)ps.vals;
  // every wavefront's key and candidate pivot value at once: all loads
  // issued before any is used (the empty asm keeps them together, one LDS
  // round trip); keys carry distinct rows, so the largest is unique
  unsigned long long kw[NW];
  T vw[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    kw[w] = ps.key[s0 + w];
    vw[w] = vals[(s0 + w) * 16 + C];
  }
  asm volatile("" ::: "memory");
  unsigned long long best = kw[0];
  T pval = vw[0];
  int bw = 0;
#pragma unroll
  for (int w = 1; w < NW; ++w) {
    if (kw[w] > best) {
      best = kw[w];
      pval = vw[w];
      bw = w;
    }
  }
  // at least 16 - C rows are active, so the key names a valid row; the
  // clamp only guards the memory access
  const int bi = 0x7fffffff - (int)(unsigned)(best & 0xffffffffu);
  const int pr = (bi >= 0 && bi < R) ? bi : R - 1;
  const T *prow = vals + (s0 + bw) * 16;
  if (tid == 0) {
    pv[C] = pr;
    rst[pr] = k;
    if (pval == T(0) && *zeroPiv == 0) *zeroPiv = k * 16 + C + 1;
  }
  const T inv = (pval != T(0)) ? T(1) / pval : T(0);
  bool upd[RPT];
  T l[RPT];
#pragma unroll
  for (int h = 0; h < RPT; ++h) {
    const bool mine = tid + h * NT == pr;
    upd[h] = act[h] && !mine;
    if (mine) act[h] = false;
    l[h] = v[h][C] * inv;
    if (upd[h]) v[h][C] = l[h];
  }
#pragma unroll
  for (int cc = C + 1; cc < 16; ++cc) {
    const T u = prow[cc];
#pragma unroll
    for (int h = 0; h < RPT; ++h)
      if (upd[h]) v[h][cc] -= l[h] * u;
  }
  if constexpr (C + 1 < 16) preg_publish<T, NT, RPT, C + 1>(v, act, tid, ps);
  __syncthreads();
}

template <typename T, int NT, int RPT, int... Cs>
__device__ __forceinline__ void preg_columns(T (&v)[RPT][16], bool (&act)[RPT], int tid, int R,
                                             int k, int *pv, int *rst, int *zeroPiv,
                                             const PanelSlots &ps,
                                             std::integer_sequence<int, Cs...>) {
  (preg_column<T, NT, RPT, Cs>(v, act, tid, R, k, pv, rst, zeroPiv, ps), ...);
}

template <typename T, int NT, int RPT>
__device__ __forceinline__ void panel_wg_regs(T *P, int R, int k, int *pv, int *rst, int *zeroPiv,
                                              const PanelSlots &ps) {
  const int tid = threadIdx.x;
  T v[RPT][16];
  bool act[RPT];
#pragma unroll
  for (int h = 0; h < RPT; ++h) {
    const int r = tid + h * NT;
    act[h] = r < R && rst[r] == kInfoActive;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) v[h][cc] = r < R ? P[r * kPST + cc] : T(0);
  }
  preg_publish<T, NT, RPT, 0>(v, act, tid, ps);
  __syncthreads();
  preg_columns<T, NT, RPT>(v, act, tid, R, k, pv, rst, zeroPiv, ps,
                           std::make_integer_sequence<int, 16>());
#pragma unroll
  for (int h = 0; h < RPT; ++h) {
    const int r = tid + h * NT;
    if (r < R) {
#pragma unroll
      for (int cc = 0; cc < 16; ++cc) P[r * kPST + cc] = v[h][cc];
    }
  }
  __syncthreads();
}

// Workgroup barrier ordering LDS accesses only: global loads still in flight
// (the next step's prefetched operands) are not waited for, as they would be
// by __syncthreads().
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// factor_ll: left-looking blocked LU with partial pivoting, one workgroup
// per leaf, one block column of KT column tiles (16 KT columns) at a time
// held in the accumulator registers of the workgroup: wavefront w owns the
// row tiles w, w + NW, ... of the block column.
//
// The rows are kept in their pivot order ("positions"): after block column
// J the pivots of its panels take the positions 16 k ... 16 k + 15 (panel
// k, pivot order), the rows they displace take the pivots' old positions,
// and later block columns are formed with their rows in that order.  So
// when a block column takes the update of an earlier panel j, the rows that
// need it are exactly the positions from 16 (j + 1) on (no padding work on
// rows retired earlier), and the update is
//   U_j = L11_j^{-1} (rows 16 j ... 16 j + 15 of the block column)
//   rows from 16 (j + 1) on:  -= L21_j U_j
// with L21_j read from the work matrix (rows gathered through the position
// table) and L11_j^{-1} stored per panel beside the work matrix.  Each
// block column is formed from the operator directly (never read back), the
// earlier multipliers are read but never rewritten, and the block column is
// written once.  Its own panels are then factored: each panel goes to LDS,
// is eliminated with partial pivoting over the positions not yet retired
// (the largest magnitude, ties to the lowest position), and updates the
// block column's later tiles.  The result is the stored form of k_factor
// (multipliers in the panel columns, U rows in the pivot rows, pivot lists
// and retire steps, all indexed by the original rows), so the solves read
// it unchanged; the right-hand-side columns are block columns too, so the
// forward elimination happens on the way.
// ---------------------------------------------------------------------------
// Elements of the LDS panel buffer of k_factor_ll: a panel of R rows, or
// during the updates from earlier panels each wavefront's slots for the
// coming step's multipliers (RTW 16 x 16 tiles per wavefront).
__host__ __device__ constexpr size_t ll_panel_elems(int R, int NW, int RTW) {
  return (size_t)R * kPST > (size_t)NW * RTW * 256 ? (size_t)R * kPST : (size_t)NW * RTW * 256;
}

template <typename T, int NW, int RTW, int KT, int MINB>
__global__ void __launch_bounds__(64 * NW, MINB) k_factor_ll(Geom g, T *M, int *piv, int *rstep,
                                                            int *info, Sel sel, BuildSrc bs) {
  constexpr int NT = 64 * NW;
  constexpr int KW = 16 * KT;
  using Acc = typename Mfma<T>::acc;
  extern __shared__ __align__(16) unsigned char smem[];
  const int wi = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int leaf;
  if (!resolve_leaf(sel, leaf)) return;
  const int R = g.R, RT = g.RT, CT = g.CT;
  T *P = (T *)smem;                          // [R][kPST]  panel, rows = positions - 16 c0
  T *Abuf = P;                               // [NW][RTW][256] (shares P: updates only)
  T *Ub = P + ll_panel_elems(R, NW, RTW);    // [2][16][KW] U rows
  T *Lk = Ub + 2 * 16 * KW;                  // [16][kPST] L11^{-1} of the current panel
  T *redv = Lk + 16 * kPST;                  // [2][NW]
  int *ord = (int *)(redv + 2 * NW);         // [R] position -> row
  int *where = ord + R;                      // [R] row -> position
  int *pst = where + R;                      // [R] (position - 16 c0) -> panel that retired it
  int *prow = pst + R;                       // [R] (position - 16 c0) -> index in its panel's pivots
  int *pvs = prow + R;                       // [KT][16] pivots of this block column's panels
  int *redi = pvs + 16 * KT;                 // [2][NW]
  int *zeroPiv = redi + 2 * NW;              // [1]
  T *Ml = M + leaf_stride(g) * wi;
  T *Lg = Ml + work_elems(g);                // [RT][16][16] L11^{-1} of every panel
  const LeafScale sc = leaf_scale(g, leaf);
  const int lr = lane >> 4, lc = lane & 15;

  for (int r = tid; r < R; r += NT) {
    ord[r] = r;
    where[r] = r;
  }
  if (tid == 0) *zeroPiv = 0;
  __syncthreads();

  Acc acc[RTW][KT];
  const int nblk = (CT + KT - 1) / KT;
  for (int J = 0; J < nblk; ++J) {
    const int c0 = J * KT;
    const int ncol = min(KT, CT - c0);          // column tiles in the block
    const int npan = max(0, min(KT, RT - c0));  // pivot panels in the block
    const int nprev = min(c0, RT);              // earlier pivot panels

    // the block column from the operator, rows in position order: one
    // column tile at a time through LDS (a rolled loop, not KT x RTW x 4
    // inlined operator evaluations), then into the registers
#pragma unroll
    for (int c = 0; c < KT; ++c) {
      if (c < ncol) {
        const int col0 = 16 * (c0 + c);
        if (build_tile_sparse(g, bs, col0)) {
          // the operator's columns reach only the grid lines through their
          // node: zeros first, then the padding rows' identity and the line
          // entries at their rows' positions
          for (int e = tid; e < R * 16; e += NT) P[(e >> 4) * kPST + (e & 15)] = T(0);
          __syncthreads();
          if (tid < 16 && col0 + tid >= g.ni && col0 + tid < R)
            P[where[col0 + tid] * kPST + tid] = T(1);
          const int per = 2 * g.m - 1;
          for (int e = tid; e < 16 * per; e += NT) {
            const int cc = e / per, q = e - cc * per;
            int i, j, k, l;
            if (line_entry(g, bs, col0 + cc, q, i, j, k, l)) {
              const int r = (j - 1) * g.m + (i - 1);
              P[where[r] * kPST + cc] =
                  (T)opval(g, g.D, g.D2, sc, (size_t)leaf * g.p * g.p, i, j, k, l);
            }
          }
        } else {
          for (int e = tid; e < R * 16; e += NT) {
            const int pos = e >> 4, cc = e & 15;
            P[pos * kPST + cc] = (T)build_elem(g, sc, leaf, bs, ord[pos], 16 * (c0 + c) + cc);
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < RTW; ++i) {
        const int t = wv + NW * i;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          acc[i][c][q] = (t < RT && c < ncol) ? (double)P[(16 * t + Tile<T>::crow(q, lane)) * kPST + lc]
                                              : 0.0;
      }
      __syncthreads();
    }

    // U rows of tile j (the pivots of panel j, in pivot order) from its
    // current values, by the wavefront that owns the tile, into the LDS
    // buffer `buf` where the others read them.  The tile's accumulators are
    // the B operand as they stand: register kc holds row 4 kc + lr, the
    // index L11^{-1} (the A operand) is paired with.
    auto make_u = [&](int j, T *buf, const T (&a)[4]) {
#pragma unroll
      for (int i = 0; i < RTW; ++i) {
        if (wv + NW * i != j) continue;
        Acc u[KT];
#pragma unroll
        for (int c = 0; c < KT; ++c) {
#pragma unroll
          for (int q = 0; q < 4; ++q) u[c][q] = 0.0;
          if (c < ncol) {
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) u[c] = Mfma<T>::op(a[kc], (T)acc[i][c][kc], u[c]);
          }
        }
#pragma unroll
        for (int c = 0; c < KT; ++c) {
          if (c < ncol) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              buf[Tile<T>::crow(q, lane) * KW + 16 * c + lc] = (T)u[c][q];
              acc[i][c][q] = (double)(T)u[c][q];
            }
          }
        }
      }
    };
    // multipliers of panel j for the rows of tile t = wv + NW i, gathered
    // through the positions straight into this wavefront's LDS slot i
    // (global-to-LDS loads: no registers held while they are in flight; each
    // lane's 16 bytes land at the slot base + 16 lane, i.e. the tile in
    // row-major order).  The positions do not move during the updates, so
    // each lane's source offsets (row part) are formed once per block column.
    constexpr int kPer = 1024 / (int)sizeof(T);   // elements per instruction
    constexpr int kIns = 256 / kPer;               // instructions per tile
    int roff[RTW][kIns];
#pragma unroll
    for (int i = 0; i < RTW; ++i) {
      const int t = min(wv + NW * i, RT - 1);
#pragma unroll
      for (int h = 0; h < kIns; ++h) {
        const int e = h * kPer + lane * (16 / (int)sizeof(T));
        const int row = ord[16 * t + (e >> 4)];
        roff[i][h] = (int)tix<T>(row, e & 15, CT);
      }
    }
    auto dma_a = [&](int i, int j) {
      T *dst = Abuf + (size_t)(wv * RTW + i) * 256;
#pragma unroll
      for (int h = 0; h < kIns; ++h) {
        const T *src = Ml + roff[i][h] + (size_t)j * 256;
        __builtin_amdgcn_global_load_lds((const void *)src,
                                         (__attribute__((address_space(3))) void *)(dst + h * kPer),
                                         16, 0, 0);
      }
    };
    // the A operand of tile i from its slot.  In MFMA step kc lane group lr
    // contracts over index 4 lr + kc (the same pairing in B), so a lane reads
    // four consecutive values.
    auto read_a = [&](int i, T (&a)[4]) {
      const T *src = Abuf + (size_t)(wv * RTW + i) * 256 + lc * 16 + 4 * lr;
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) a[kc] = src[kc];
    };
    // tile i takes step j's update (b holds -U); its slot then refills with
    // panel jn's multipliers (when the tile needs them), so that load is in
    // flight during the rest of the step.  The empty asm consumes the A
    // operand before the refill: the slot's reads have completed, and no
    // memory operation moves above it.
    auto mma = [&](int i, const T (&b)[KT][4], int jn) {
      T a[4];
      read_a(i, a);
#pragma unroll
      for (int c = 0; c < KT; ++c) {
        if (c < ncol) {
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) acc[i][c] = Mfma<T>::op(a[kc], b[c][kc], acc[i][c]);
        }
      }
      if (jn >= 0 && wv + NW * i > jn) {
        asm volatile("" ::"v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]) : "memory");
        dma_a(i, jn);
      }
    };

    // updates from the earlier panels, in order.  Each step's multipliers
    // are loaded into LDS a step ahead (and the L11^{-1} the next U needs
    // into registers); the barrier orders LDS only, so those loads stay in
    // flight across it and each wavefront waits only for its own.  The
    // owner of tile j + 1 takes step j there first and forms U_{j+1} before
    // the next barrier.
    T lpre[4];
    if (nprev > 0) {
#pragma unroll
      for (int i = 0; i < RTW; ++i) {
        const int t = wv + NW * i;
        if (t > 0 && t < RT) dma_a(i, 0);
      }
      if (wv == 0) {
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) lpre[kc] = Lg[lc * 16 + 4 * kc + lr];
        make_u(0, Ub, lpre);
      }
      if (nprev > 1 && wv == 1 % NW) {
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) lpre[kc] = Lg[256 + lc * 16 + 4 * kc + lr];
      }
    }
    for (int j = 0; j < nprev; ++j) {
      lds_barrier();
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wavefront's loads of step j
      const T *U = Ub + (j & 1) * 16 * KW;
      T b[KT][4];
#pragma unroll
      for (int c = 0; c < KT; ++c) {
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) b[c][kc] = c < ncol ? -U[(4 * lr + kc) * KW + 16 * c + lc] : T(0);
      }
      const int jn = j + 1;
      const int jload = jn < nprev ? jn : -1;
      const bool ahead = jn < nprev && wv == jn % NW;
      if (ahead) {
#pragma unroll
        for (int i = 0; i < RTW; ++i)
          if (wv + NW * i == jn) mma(i, b, jload);
      }
#pragma unroll
      for (int i = 0; i < RTW; ++i) {
        const int t = wv + NW * i;
        if (t > j && t < RT && !(ahead && t == jn)) mma(i, b, jload);
      }
      // U_{j+1} last: tile j+1's products have long completed by then, so
      // forming it stalls nothing
      if (ahead) make_u(jn, Ub + (jn & 1) * 16 * KW, lpre);
      if (jn < nprev) {
        if (jn + 1 < nprev && wv == (jn + 1) % NW) {
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) lpre[kc] = Lg[(jn + 1) * 256 + lc * 16 + 4 * kc + lr];
        }
      }
    }
    __syncthreads();

    // the rows retired by earlier block columns (positions below 16 c0) now
    // hold their final U values: out at once, so that the panel tile's
    // registers are free while its panel is eliminated
#pragma unroll
    for (int i = 0; i < RTW; ++i) {
      const int t = wv + NW * i;
      if (t >= c0 || t >= RT) continue;
#pragma unroll
      for (int c = 0; c < KT; ++c) {
        if (c >= ncol) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = ord[16 * t + Tile<T>::crow(q, lane)];
          Ml[tix<T>(row, 16 * (c0 + c) + lc, CT)] = (T)acc[i][c][q];
        }
      }
    }

    // this block column's own panels, in turn.  The panel being factored is
    // always register tile 0: after each panel the block column's tiles
    // rotate by one, KT times in all, so that every register index stays a
    // compile-time constant and the tiles end in their order again.
    if (npan > 0) {
      const int Rr = R - 16 * c0;
      for (int r = tid; r < Rr; r += NT) pst[r] = kInfoActive;
      __syncthreads();
#pragma unroll 1
      for (int s = 0; s < KT; ++s) {
        if (s < npan) {
          const int k = c0 + s;
          int *pv = pvs + 16 * s;
#pragma unroll
          for (int i = 0; i < RTW; ++i) {
            const int t = wv + NW * i;
            if (t >= c0 && t < RT) {
#pragma unroll
              for (int q = 0; q < 4; ++q)
                P[(16 * (t - c0) + Tile<T>::crow(q, lane)) * kPST + lc] = (T)acc[i][0][q];
            }
          }
          __syncthreads();
          if constexpr (NW == 4) {
            if (wv == 0) {
              panel_one_wave<T>(P, Rr, k, lane, pv, pst, zeroPiv);
              wave_lds_fence<T>();
            }
          } else {
            // the panel's slots in the U-row buffer (free until the panel is done)
            static_assert(16 * NW * RTW <= 64 * NW * ((RTW + 3) / 4), "panel rows per thread");
            PanelSlots ps;
            ps.key = (unsigned long long *)Ub;
            ps.vals = (void *)(ps.key + 2 * NW);
            panel_wg_regs<T, NT, (RTW + 3) / 4>(P, Rr, k, pv, pst, zeroPiv, ps);
          }
          if (wv == 0) {
            linv16<T>(P, pv, Lk, lane);
            if (lane < 16) prow[pv[lane]] = lane;
            wave_lds_fence<T>();
            if (lane < 16) {
#pragma unroll
              for (int r = 0; r < 16; ++r) Lg[k * 256 + r * 16 + lane] = Lk[r * kPST + lane];
            }
          }
          __syncthreads();
#pragma unroll
          for (int i = 0; i < RTW; ++i) {
            const int t = wv + NW * i;
            const bool live = t >= c0 && t < RT;
#pragma unroll
            for (int q = 0; q < 4; ++q)
              acc[i][0][q] = live ? (double)P[(16 * max(t - c0, 0) + Tile<T>::crow(q, lane)) * kPST + lc]
                                  : 0.0;
          }
          if (s + 1 < ncol) {
            // raw pivot rows of the block's later column tiles (register
            // tiles 1, 2, ...) into Ub, U = L11^{-1} of them in place, then
            // pivot rows take U and the rows still active take -L21 U (L21
            // from the panel in LDS)
#pragma unroll
            for (int i = 0; i < RTW; ++i) {
              const int t = wv + NW * i;
              if (t >= c0 && t < RT) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  const int rp = 16 * (t - c0) + Tile<T>::crow(q, lane);
                  if (pst[rp] == k) {
                    const int c = prow[rp];
#pragma unroll
                    for (int sp = 1; sp < KT; ++sp)
                      if (s + sp < ncol) Ub[c * KW + 16 * sp + lc] = (T)acc[i][sp][q];
                  }
                }
              }
            }
            __syncthreads();
            for (int sp = 1 + wv; s + sp < ncol; sp += NW) {
              const Acc u = tri_apply<T>(Lk, Ub, KW, 16 * sp, lane);
              wave_lds_fence<T>();
#pragma unroll
              for (int q = 0; q < 4; ++q) Ub[Tile<T>::crow(q, lane) * KW + 16 * sp + lc] = (T)u[q];
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < RTW; ++i) {
              const int t = wv + NW * i;
              if (t < c0 || t >= RT) continue;
              const int ra = 16 * (t - c0) + lc;
              const bool act = pst[ra] == kInfoActive;
              T a[4];
#pragma unroll
              for (int kc = 0; kc < 4; ++kc) a[kc] = act ? -P[ra * kPST + 4 * kc + lr] : T(0);
#pragma unroll
              for (int sp = 1; sp < KT; ++sp) {
                if (s + sp >= ncol) continue;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  const int rp = 16 * (t - c0) + Tile<T>::crow(q, lane);
                  if (pst[rp] == k) acc[i][sp][q] = (double)Ub[prow[rp] * KW + 16 * sp + lc];
                }
#pragma unroll
                for (int kc = 0; kc < 4; ++kc)
                  acc[i][sp] = Mfma<T>::op(a[kc], Ub[(4 * kc + lr) * KW + 16 * sp + lc], acc[i][sp]);
              }
            }
          }
          __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < RTW; ++i) {
          const Acc first = acc[i][0];
#pragma unroll
          for (int c = 0; c + 1 < KT; ++c) acc[i][c] = acc[i][c + 1];
          acc[i][KT - 1] = first;
        }
      }
    }

    // the rest of the block column, once, at the rows' places in the work
    // matrix
#pragma unroll
    for (int i = 0; i < RTW; ++i) {
      const int t = wv + NW * i;
      if (t < c0 || t >= RT) continue;
#pragma unroll
      for (int c = 0; c < KT; ++c) {
        if (c >= ncol) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = ord[16 * t + Tile<T>::crow(q, lane)];
          Ml[tix<T>(row, 16 * (c0 + c) + lc, CT)] = (T)acc[i][c][q];
        }
      }
    }

    // the pivots of this block column take the positions 16 k + c; the rows
    // they displace (those at the targets that are not pivots) take the
    // pivots' places outside the targets, the n-th displaced row the n-th
    // such place.  One wavefront, lane e moving pivot e.
    if (npan > 0) {
      if (wv == 0) {
        const int nt = 16 * npan;
        const bool on = lane < nt;
        const int rel = on ? pvs[lane] : 0;               // pivot's position - 16 c0
        const int row = on ? ord[16 * c0 + rel] : 0;
        const int cur = on ? ord[16 * c0 + lane] : 0;     // the row at the target now
        const bool disp = on && pst[lane] == kInfoActive;
        const bool frees = on && rel >= nt;
        const unsigned long long dm = __ballot(disp), fm = __ballot(frees);
        const unsigned long long below = (1ull << lane) - 1ull;
        int *moved = (int *)Ub;                            // free until the next block column
        if (disp) moved[__popcll(dm & below)] = cur;
        wave_lds_fence<T>();
        if (on) {
          ord[16 * c0 + lane] = row;
          where[row] = 16 * c0 + lane;
          piv[(size_t)wi * R + 16 * c0 + lane] = row;
          rstep[(size_t)wi * R + row] = c0 + lane / 16;
        }
        if (frees) {
          const int other = moved[__popcll(fm & below)];
          ord[16 * c0 + rel] = other;
          where[other] = 16 * c0 + rel;
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) info[leaf] = *zeroPiv;
}

// ---------------------------------------------------------------------------
// factor_rr: the same factorisation with the whole FP32 work matrix held in
// registers (R <= 208, i.e. p <= 16: 13 x 17 tiles, 226 KB per leaf, spread
// over the register files of one CU), so that no trailing tile travels
// through L2/HBM; one workgroup of NW wavefronts per leaf.  Wavefront w owns
// the column tiles w, w + NW, ... (all row tiles of each), as FP32 values in
// the FP64 MFMA accumulator order (lane l: column l%16, rows 4q + l/16).
// Panel k is factored by the owner of column tile k with the
// single-wavefront panel, into one of two LDS buffers, together with
// L11^{-1}.  Step k then updates every column tile right of k: the 16 pivot
// rows are gathered (the rows a lane holds are the same in every column
// tile, so a per-lane mask of "my rows retired at step k" selects them),
// U12 = L11^{-1} A12 is formed on MFMA and put back into the pivot rows, and
// the active row tiles take C -= L21 U12, four row tiles at a time.  Look-
// ahead: within step k the owner of column tile k+1 updates that tile
// first and factors panel k+1 into the other buffer while the remaining
// updates of step k proceed, so the serial panel overlaps the MFMA work.
// (Rows retired by panel k+1 are still "after k" for step k: the update
// mask is rstep > k.)  The result is the stored form of k_factor
// (multipliers in the panel columns, U rows in the pivot rows, retire
// steps), written to the work matrix once at the end.
// ---------------------------------------------------------------------------
template <int RT, int NW, int NS>
__global__ void __launch_bounds__(64 * NW, 1) k_factor_rr(Geom g, float *M, int *piv, int *rstep,
                                                          int *info, Sel sel, BuildSrc bs) {
  constexpr int R = 16 * RT;
  constexpr int NT = 64 * NW;
  __shared__ float P[2][R * kPST];           // panels (double-buffered); build staging
  __shared__ float Li[2][16 * kPST];         // L11^{-1} of each panel buffer
  __shared__ float Ub[NW][17 * kPST];        // per wavefront: pivot rows, then U12 (+ trash row)
  __shared__ float prb[16];                  // pivot row broadcast inside a panel
  __shared__ int rst[R];
  __shared__ int prow[R];                    // position of a pivot row in its panel's pv
  __shared__ int pvs[2][16];
  __shared__ int tileAct[2][RT], tilePiv[2][RT];
  __shared__ int zeroPiv;
  __shared__ double tab[7 * 256];            // D, D^2 and the leaf's coefficient samples (p <= 16)
  const int wi = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int leaf;
  if (!resolve_leaf(sel, leaf)) return;
  const int CT = g.CT, p = g.p, pp = p * p, m = g.m, ni = g.ni, nb = g.nb;
  const int lr = lane >> 4, lc = lane & 15;
  float v[NS][RT][4];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int ti = 0; ti < RT; ++ti)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[s][ti][q] = 0.0f;
  {
    // stage the tables, then build W one column tile at a time through LDS
    auto stage = [&](const double *src, int slot, bool per_leaf) -> const double * {
      if (!src) return nullptr;
      const double *sp = per_leaf ? src + (size_t)leaf * pp : src;
      for (int e = tid; e < pp; e += NT) tab[slot * 256 + e] = sp[e];
      return tab + slot * 256;
    };
    StagedOp t;
    t.D = stage(g.D, 0, false);
    t.D2 = stage(g.D2, 1, false);
    t.a11 = stage(g.a11, 2, true);
    t.c1 = stage(g.c1, 3, true);
    t.a22 = stage(g.a22, 4, true);
    t.c2 = stage(g.c2, 5, true);
    t.k2b = stage(g.k2b, 6, true);
    __syncthreads();
    const LeafScale sc = leaf_scale(g, leaf);
    // this thread's column within a tile and first row; rows step by NT/16
    constexpr int RSTEP = NT / 16;
    const int cc = tid & 15, r0 = tid >> 4;
    const int i0 = r0 % m + 1, j0 = r0 / m + 1;
    float *P0 = P[0];
    for (int J = 0; J < CT; ++J) {
      const int c = 16 * J + cc;
      int kind = 4, kc = 0, lcn = 0;   // 0 interior node, 2 boundary node, 3 f, 4 zero
      if (c < ni) {
        kind = 0;
        kc = c % m + 1;
        lcn = c / m + 1;
      } else if (c >= R) {
        const int jr = c - R;
        if (jr < nb) {
          kind = 2;
          bnode(jr, m, p, kc, lcn);
        } else if (jr == nb && bs.f) {
          kind = 3;
        }
      }
      int i = i0, jj = j0;
      for (int r = r0; r < R; r += RSTEP) {
        float val = 0.0f;
        if (r >= ni) {
          val = (c == r) ? 1.0f : 0.0f;
        } else if (kind <= 2) {
          val = (float)opval_s(p, t, sc, i, jj, kc, lcn);
        } else if (kind == 3) {
          val = (float)bs.f[(size_t)leaf * ni + r];
        }
        P0[r * kPST + cc] = val;
        i += RSTEP;
        while (i > m) {
          i -= m;
          ++jj;
        }
      }
      __syncthreads();
      if (wv == J % NW) {
        const int sj = J / NW;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          if (s == sj) {
#pragma unroll
            for (int ti = 0; ti < RT; ++ti)
#pragma unroll
              for (int q = 0; q < 4; ++q) v[s][ti][q] = P0[(16 * ti + 4 * q + lr) * kPST + lc];
          }
        }
      }
      __syncthreads();
    }
  }
  for (int r = tid; r < R; r += NT) rst[r] = kInfoActive;
  int zp = 0;   // first zero pivot (1-based column) seen by this wavefront's panels
  __syncthreads();

  // k = -1 only factors panel 0; step k >= 0 updates with panel k and, in
  // the wavefront owning column tile k+1, factors panel k+1 on the way.
  for (int k = -1; k < RT; ++k) {
    const int b = k & 1;
    unsigned ta = 0, tp = 0;
    unsigned long long pm = 0;
    if (k >= 0) {
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        ta |= (unsigned)(tileAct[b][t] != 0) << t;
        tp |= (unsigned)(tilePiv[b][t] != 0) << t;
      }
      ta = __builtin_amdgcn_readfirstlane(ta);
      tp = __builtin_amdgcn_readfirstlane(tp);
#pragma unroll
      for (int ti = 0; ti < RT; ++ti) {
        if ((tp >> ti) & 1u) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (rst[16 * ti + 4 * q + lr] == k) pm |= 1ull << (4 * ti + q);
        }
      }
    }
    const int kn = k + 1, sn = kn / NW;
    const bool owner_next = kn < RT && wv == kn % NW;
    const float *Pk = P[b];
    const float *Lk = Li[b];
    float *U = Ub[wv];
    // pass 0: the next panel's column tile (its owner only), then that
    // panel; pass 1: every other column tile right of k
    for (int pass = 0; pass < 2; ++pass) {
      if (k >= 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const int j = wv + NW * s;
          if (j >= CT || j <= k) continue;
          if ((pass == 0) != (owner_next && s == sn)) continue;
          // pivot rows into U (rows of other lanes go to the trash row 16)
#pragma unroll
          for (int ti = 0; ti < RT; ++ti) {
            if ((tp >> ti) & 1u) {
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const bool isp = (pm >> (4 * ti + q)) & 1ull;
                const int d = isp ? prow[16 * ti + 4 * q + lr] : 16;
                U[d * kPST + lc] = v[s][ti][q];
              }
            }
          }
          wave_lds_fence<float>();
          const d4 u = tri_apply<float>(Lk, U, kPST, 0, lane);
          wave_lds_fence<float>();
#pragma unroll
          for (int q = 0; q < 4; ++q) U[(4 * q + lr) * kPST + lc] = (float)u[q];
          wave_lds_fence<float>();
#pragma unroll
          for (int ti = 0; ti < RT; ++ti) {
            if ((tp >> ti) & 1u) {
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const bool isp = (pm >> (4 * ti + q)) & 1ull;
                const float w = U[(isp ? prow[16 * ti + 4 * q + lr] : 16) * kPST + lc];
                v[s][ti][q] = isp ? w : v[s][ti][q];
              }
            }
          }
          float bop[4];
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) bop[kc] = U[(4 * kc + lr) * kPST + lc];
          // C -= L21 U12 on the active row tiles, four independent tiles at a time
#pragma unroll
          for (int tg = 0; tg < (RT + 3) / 4; ++tg) {
            if (!((ta >> (4 * tg)) & 0xfu)) continue;
            constexpr int G = 4;
            float a[G][4];
            d4 c[G];
#pragma unroll
            for (int tt = 0; tt < G; ++tt) {
              const int ti = 4 * tg + tt;
              if (ti >= RT) continue;
              const int ar = 16 * ti + lc;
              const bool act = rst[ar] > k;
#pragma unroll
              for (int kc = 0; kc < 4; ++kc) a[tt][kc] = act ? -Pk[ar * kPST + 4 * kc + lr] : 0.0f;
#pragma unroll
              for (int q = 0; q < 4; ++q) c[tt][q] = v[s][ti][q];
            }
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
#pragma unroll
              for (int tt = 0; tt < G; ++tt)
                if (4 * tg + tt < RT) c[tt] = Mfma<float>::op(a[tt][kc], bop[kc], c[tt]);
            }
#pragma unroll
            for (int tt = 0; tt < G; ++tt) {
              const int ti = 4 * tg + tt;
              if (ti >= RT) continue;
#pragma unroll
              for (int q = 0; q < 4; ++q) v[s][ti][q] = (float)c[tt][q];
            }
          }
          wave_lds_fence<float>();
        }
      }
      if (pass == 0 && owner_next) {
        // factor panel kn into buffer kn & 1
        const int bn = kn & 1;
        float *Pn = P[bn];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          if (s == sn) {
#pragma unroll
            for (int ti = 0; ti < RT; ++ti)
#pragma unroll
              for (int q = 0; q < 4; ++q) Pn[(16 * ti + 4 * q + lr) * kPST + lc] = v[s][ti][q];
          }
        }
        wave_lds_fence<float>();
        {
          float pr[4][16];
          unsigned act = 0;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int r = lane + 64 * t;
            const bool in = r < R;
            if (in && rst[r] == kInfoActive) act |= 1u << t;
#pragma unroll
            for (int c = 0; c < 16; ++c) pr[t][c] = in ? Pn[r * kPST + c] : 0.0f;
          }
          rr_panel_columns(pr, act, lane, kn, prb, pvs[bn], rst, zp,
                           std::make_integer_sequence<int, 16>());
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int r = lane + 64 * t;
            if (r < R) {
#pragma unroll
              for (int c = 0; c < 16; ++c) Pn[r * kPST + c] = pr[t][c];
            }
          }
        }
        wave_lds_fence<float>();
        linv16<float>(Pn, pvs[bn], Li[bn], lane);
        if (lane < 16) {
          prow[pvs[bn][lane]] = lane;
          piv[(size_t)wi * R + kn * 16 + lane] = pvs[bn][lane];
        }
        for (int t = lane; t < RT; t += 64) {
          int ac = 0, pc = 0;
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const int st = rst[t * 16 + q];
            ac |= (st == kInfoActive);
            pc |= (st == kn);
          }
          tileAct[bn][t] = ac;
          tilePiv[bn][t] = pc;
        }
        wave_lds_fence<float>();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          if (s == sn) {
#pragma unroll
            for (int ti = 0; ti < RT; ++ti)
#pragma unroll
              for (int q = 0; q < 4; ++q) v[s][ti][q] = Pn[(16 * ti + 4 * q + lr) * kPST + lc];
          }
        }
      }
    }
    __syncthreads();
  }

  float *Ml = M + leaf_stride(g) * wi;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int j = wv + NW * s;
    if (j >= CT) continue;
#pragma unroll
    for (int ti = 0; ti < RT; ++ti)
#pragma unroll
      for (int q = 0; q < 4; ++q) Ml[((size_t)(ti * CT + j) << 8) + q * 64 + lane] = v[s][ti][q];
  }
  for (int r = tid; r < R; r += NT) rstep[(size_t)wi * R + r] = rst[r];
  // the first zero pivot over all panels (each panel owner's lane 0 saw its own)
  if (tid == 0) zeroPiv = INT_MAX;
  __syncthreads();
  if (lane == 0 && zp) atomicMin(&zeroPiv, zp);
  __syncthreads();
  if (tid == 0) info[leaf] = zeroPiv == INT_MAX ? 0 : zeroPiv;
}

// ---------------------------------------------------------------------------
// Blocked triangular solves with the stored factorisation on the right-hand
// sides held in the work matrix.  A super-step takes NB consecutive panels
// at once: their 16-row pivot blocks are gathered into LDS, solved one after
// another (the 16-column triangles one column per thread; each solved block
// immediately updates the pivot blocks of the super-step that depend on it),
// and then every remaining row of the right-hand sides receives all NB
// updates in one MFMA pass, C -= sum_b W[r, panel b] Y_b.  The right-hand
// sides therefore stream through memory once per NB panels instead of once
// per panel.  Forward (refinement only): panels ascending, unit lower L11,
// rows retired after the super-step are updated, the solved pivot rows are
// written back into the work matrix.  Backward: panels descending, U11 with
// its diagonal, rows retired before the super-step are updated, X (or h, or
// u_i) written in FP64.
// ---------------------------------------------------------------------------
constexpr int kSolveNB = 4;   // panels per super-step

// C -= sum over the nbk blocks of W[r, panel pb[i]] * Yb[i] on the row tiles
// flagged in tileAny, for rows retired after kmax (after) or before kmin.
template <typename T, int NW>
__device__ __forceinline__ void strip_update_nb(T *Ml, const T *Y, int YST, const int *rst,
                                                const int *tileAny, int RT, int CT, int R,
                                                int ntj, int k0, int nbk, int dir, bool after,
                                                int kbound, int wv, int lane) {
  const int nstrip = (ntj + 3) >> 2;
  const int nall = RT * nstrip;
  for (int t = wv; t < nall; t += NW) {
    const int ti = t / nstrip;
    if (!tileAny[ti]) continue;
    const int j0 = (t - ti * nstrip) * 4;
    const int nj = min(4, ntj - j0);
    T *Ct = Ml + ((size_t)(ti * CT + (R >> 4) + j0) << 8);
    const int ar = ti * 16 + (lane & 15);
    const bool use = after ? rst[ar] > kbound : rst[ar] < kbound;
    typename Mfma<T>::acc c[4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      if (jj < nj) {
#pragma unroll
        for (int q = 0; q < 4; ++q) c[jj][q] = Ct[jj * 256 + q * 64 + lane];
      }
    }
#pragma unroll 1
    for (int i = 0; i < nbk; ++i) {
      const int pb = k0 + dir * i;
      T a[4];
#pragma unroll
      for (int kc = 0; kc < 4; ++kc)
        a[kc] = use ? -Ml[tix<T>(ar, pb * 16 + 4 * kc + (lane >> 4), CT)] : T(0);
      const T *Yb = Y + (size_t)i * 16 * YST;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        if (jj < nj) {
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) {
            const T bq = Yb[(4 * kc + (lane >> 4)) * YST + (j0 + jj) * 16 + (lane & 15)];
            c[jj] = Mfma<T>::op(a[kc], bq, c[jj]);
          }
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      if (jj < nj) {
#pragma unroll
        for (int q = 0; q < 4; ++q) Ct[jj * 256 + q * 64 + lane] = (T)c[jj][q];
      }
    }
  }
}

// PASSES: 1 backward only, 2 forward only, 3 forward then backward (the
// refinement correction in one launch).
template <typename T, int NT, int PASSES>
__global__ void __launch_bounds__(NT) k_trisolve(Geom g, T *M, const int *piv, const int *rstep,
                                                 BackOut o, Sel sel, int CW) {
  constexpr int NW = NT / 64, NB = kSolveNB;
  extern __shared__ __align__(16) unsigned char smem[];
  const int wi = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int leaf;
  if (!resolve_leaf(sel, leaf)) return;
  if (o.skip && o.skip[leaf]) return;
  const int R = g.R, RT = g.RT, CT = g.CT, ni = g.ni, nb = g.nb;
  // this workgroup's right-hand-side columns: [c0, c0 + NRC) of the CW-wide
  // chunk blockIdx.y (whole 16-column tiles)
  const int c0 = blockIdx.y * CW, NRC = min(CW, CT * 16 - R - c0), YST = CW + 16;
  double *red = (double *)smem;     // [NW]
  T *Y = (T *)(red + NW);           // [NB][16][YST] pivot blocks of the super-step
  T *Tt = Y + NB * 16 * YST;        // [16][kPST] triangle of the current panel
  T *Td = Tt + 16 * kPST;           // [16] reciprocals of its diagonal (backward)
  T *Tx = Td + 16;                  // [NB][16][kPST] couplings to the later blocks
  int *rst = (int *)(Tx + NB * 16 * kPST);
  int *tileAny = rst + R;
  int *pva = tileAny + RT;          // [R] all pivots of the leaf
  T *Ml = M + leaf_stride(g) * wi;
  double nd = 0.0;
  for (int r = tid; r < R; r += NT) {
    rst[r] = rstep[(size_t)wi * R + r];
    pva[r] = piv[(size_t)wi * R + r];
  }
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
  const bool FWD = pass == 0;
  if (!(PASSES & (FWD ? 2 : 1))) continue;
  const int dir = FWD ? 1 : -1;
  for (int k0 = FWD ? 0 : RT - 1; FWD ? k0 < RT : k0 >= 0; k0 += dir * NB) {
    const int nbk = FWD ? min(NB, RT - k0) : min(NB, k0 + 1);
    const int klast = k0 + dir * (nbk - 1);
    // gather the pivot blocks of the super-step; flag the row tiles that the
    // closing update touches
    for (int e = tid; e < nbk * 16 * NRC; e += NT) {
      const int i = e / (16 * NRC), rem = e - i * 16 * NRC, s = rem / NRC, jr = rem - s * NRC;
      Y[(i * 16 + s) * YST + jr] = Ml[tix<T>(pva[16 * (k0 + dir * i) + s], R + c0 + jr, CT)];
    }
    for (int t = tid; t < RT; t += NT) {
      int a = 0;
      for (int q = 0; q < 16; ++q) {
        const int st = rst[t * 16 + q];
        a |= FWD ? (st > klast) : (st < klast);
      }
      tileAny[t] = a;
    }
    for (int i = 0; i < nbk; ++i) {
      const int b = k0 + dir * i;
      const int *pv = pva + 16 * b;
      // triangle of panel b, and the couplings of the later pivot blocks
      // to panel b's unknowns
      for (int e = tid; e < 256; e += NT) {
        const int s = e >> 4, q = e & 15;
        const T u = Ml[tix<T>(pv[s], b * 16 + q, CT)];
        Tt[s * kPST + q] = u;
        if (!FWD && q == s) Td[s] = T(1) / u;
      }
      for (int e = tid; e < (nbk - 1 - i) * 256; e += NT) {
        const int i2 = i + 1 + (e >> 8), s2 = (e >> 4) & 15, q = e & 15;
        Tx[(i2 * 16 + s2) * kPST + q] = Ml[tix<T>(pva[16 * (k0 + dir * i2) + s2], b * 16 + q, CT)];
      }
      __syncthreads();
      for (int jr = tid; jr < NRC; jr += NT) {
        T x[16];
#pragma unroll
        for (int s = 0; s < 16; ++s) x[s] = Y[(i * 16 + s) * YST + jr];
        if (FWD) {
#pragma unroll
          for (int s = 0; s < 16; ++s) {
#pragma unroll
            for (int q = s + 1; q < 16; ++q) x[q] -= Tt[q * kPST + s] * x[s];
          }
        } else {
#pragma unroll
          for (int s = 15; s >= 0; --s) {
            x[s] *= Td[s];
#pragma unroll
            for (int q = 0; q < s; ++q) x[q] -= Tt[q * kPST + s] * x[s];
          }
        }
#pragma unroll
        for (int s = 0; s < 16; ++s) Y[(i * 16 + s) * YST + jr] = x[s];
        // the later pivot blocks of the super-step take panel b's update
#pragma unroll 1
        for (int i2 = i + 1; i2 < nbk; ++i2) {
#pragma unroll
          for (int s2 = 0; s2 < 16; ++s2) {
            T acc = Y[(i2 * 16 + s2) * YST + jr];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc -= Tx[(i2 * 16 + s2) * kPST + q] * x[q];
            Y[(i2 * 16 + s2) * YST + jr] = acc;
          }
        }
        if (FWD) {
#pragma unroll
          for (int s = 0; s < 16; ++s) Ml[tix<T>(pv[s], R + c0 + jr, CT)] = x[s];
        } else if (c0 + jr < g.nrhs) {
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            const int ii = b * 16 + s;
            if (ii >= ni) continue;
            const double v = (double)x[s];
            if (o.mode == BACK_UI) {
              o.ui[(size_t)leaf * ni + ii] = v;
            } else {
              const int col = c0 + jr;
              double *dst = (col < nb) ? o.Xt + ((size_t)leaf * nb + col) * ni + ii
                                       : o.h + (size_t)leaf * ni + ii;
              if (o.mode == BACK_STORE) {
                *dst = v;
              } else {
                *dst += v;
                nd += v * v;
              }
            }
          }
        }
      }
      __syncthreads();
    }
    strip_update_nb<T, NW>(Ml, Y, YST, rst, tileAny, RT, CT, R + c0, NRC >> 4, k0, nbk, dir,
                           FWD, klast, wv, lane);
    __syncthreads();
  }
  }
  if ((PASSES & 1) && o.mode == BACK_ACCUM) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nd += __shfl_xor(nd, off);
    if (lane == 0) red[wv] = nd;
    __syncthreads();
    if (tid == 0) {
      double a = 0.0;
      for (int w = 0; w < NW; ++w) a += red[w];
      o.norms[kNormStride * (size_t)leaf + 16 + blockIdx.y] = a;
    }
  }
}

// ---------------------------------------------------------------------------
// Back substitution for work matrices of at most 256 rows with the
// right-hand sides held in registers.  Row tile i of the right-hand sides
// (all its column tiles, in pivot (step) order) lives in the FP64 MFMA
// accumulators of wavefront i mod NW for the whole solve.  The 16 x 16
// diagonal blocks of the factors are inverted once per leaf into LDS (one
// column per thread), so every step of the block substitution is a tile
// product:
//   X_k = U_kk^{-1} (Y_k - sum_{j>k} U_kj X_j)
// where U_kj is tile j of the 16 pivot rows of panel k.  Step k: the owner
// of row tile k forms X_k and publishes it in LDS; after one barrier every
// wavefront applies it to its own row tiles.  Each factor tile is thus read
// once per leaf (by the wavefront owning its row tile) and used for every
// column tile, and the tiles of step k-1 are loaded while step k runs.  The
// right-hand sides are read once and the solution written once.  RTM bounds
// RT and NCTM the number of right-hand-side column tiles (register arrays
// are indexed statically).
// ---------------------------------------------------------------------------
constexpr int kDST = 17;   // LDS row stride of the diagonal blocks

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Pivot list of the leaf (clamped into it) and the inverted 16 x 16
// diagonal blocks of its factors, into LDS; the whole workgroup takes part.
// Block b holds L_bb^{-1} (unit lower) strictly below the diagonal (forward
// pass only) and U_bb^{-1} on and above it.
template <typename T, int PASSES>
__device__ __forceinline__ void stage_inverse_diag(const Geom &g, const T *Ml, const int *pivl,
                                                   T *D, int *pva, int tid, int NT) {
  const int R = g.R, RT = g.RT, CT = g.CT;
  for (int r = tid; r < R; r += NT) pva[r] = min(max(pivl[r], 0), R - 1);
  __syncthreads();
  // diagonal block b: element (s, q) = W[pivot row of step 16b+s][16b+q]
  for (int e = tid; e < RT * 256; e += NT) {
    const int b = e >> 8, s = (e >> 4) & 15, q = e & 15;
    D[(b * 16 + s) * kDST + q] = Ml[tix<T>(pva[16 * b + s], 16 * b + q, CT)];
  }
  __syncthreads();
  // invert in place, column j of block b per thread, whole blocks per round:
  // L_bb^{-1} (unit lower) strictly below the diagonal, then U_bb^{-1} on and
  // above it (each inverse reads only its own triangle of the block)
  for (int base = 0; base < RT * 16; base += NT) {
    const int t = base + tid, b = t >> 4, j = t & 15;
    const bool mine = t < RT * 16;
    T *Db = D + (mine ? b : 0) * 16 * kDST;
    if (PASSES & 2) {
      double zl[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double acc = (i == j) ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < i; ++q) acc -= (double)Db[i * kDST + q] * zl[q];
        zl[i] = acc;
      }
      __syncthreads();
      if (mine) {
#pragma unroll
        for (int i = 1; i < 16; ++i)
          if (i > j) Db[i * kDST + j] = (T)zl[i];
      }
    }
    double zu[16];
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double acc = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int q = i + 1; q < 16; ++q) acc -= (double)Db[i * kDST + q] * zu[q];
      zu[i] = (i <= j) ? acc / (double)Db[i * kDST + i] : 0.0;
    }
    __syncthreads();
    if (mine) {
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (i <= j) Db[i * kDST + j] = (T)zu[i];
    }
    __syncthreads();
  }

}

template <typename T, int RTM, int NCTM, int NW, int MINW>
__global__ void __launch_bounds__(64 * NW, MINW) k_solve_rr(Geom g, const T *M, const int *piv,
                                                      BackOut o, Sel sel) {
  constexpr int NT = 64 * NW, RPW = (RTM + NW - 1) / NW;
  extern __shared__ __align__(16) unsigned char smem[];
  const int wi = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int leaf;
  if (!resolve_leaf(sel, leaf)) return;
  if (o.skip && o.skip[leaf]) return;
  const int R = g.R, RT = g.RT, CT = g.CT, ni = g.ni, nb = g.nb, NCT = CT - RT;
  double *red = (double *)smem;                         // [NW]
  double *xb = red + 8;                                 // [2][NCTM][256] published X_k
  T *D = (T *)(xb + 2 * NCTM * 256);                    // [RT][16][kDST]
  int *pva = (int *)(D + (size_t)RT * 16 * kDST);       // [R] pivot rows in step order
  const T *Ml = M + leaf_stride(g) * wi;
  stage_inverse_diag<T, 1>(g, Ml, piv + (size_t)wi * R, D, pva, tid, NT);

  const int cl = lane & 15, rq = lane >> 4;
  // this wavefront's row tiles i = li*NW + wv, gathered in step order
  d4 y[RPW][NCTM];
#pragma unroll
  for (int li = 0; li < RPW; ++li) {
    const int i = li * NW + wv;
#pragma unroll
    for (int c = 0; c < NCTM; ++c) {
      if (i < RT && c < NCT) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          y[li][c][q] = (double)Ml[tix<T>(pva[16 * i + 4 * q + rq], R + 16 * c + cl, CT)];
      }
    }
  }
  // factor operand of row tile i at step k: A[r][4kc + rq] = W[pivot of 16i + r][16k + 4kc + rq],
  // kept raw (no conversion or select) so that nothing waits for the loads
  // before the step that uses them; addresses are clamped into the leaf
  auto load_a = [&](T (&a)[RPW][4], int k) __attribute__((always_inline)) {
    const int kk = min(max(k, 0), RT - 1);
#pragma unroll
    for (int li = 0; li < RPW; ++li) {
      const int pr = pva[16 * min(li * NW + wv, RT - 1) + cl];
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) a[li][kc] = Ml[tix<T>(pr, 16 * kk + 4 * kc + rq, CT)];
    }
  };
  double nd = 0.0;
  // the owner of row tile k applies the inverted diagonal block to it,
  // publishes the result in LDS and writes it out
  auto form = [&](int k) __attribute__((always_inline)) {
    const T *Db = D + k * 16 * kDST;
    double *xk = xb + (k & 1) * NCTM * 256;
#pragma unroll
    for (int li = 0; li < RPW; ++li) {
      if (li * NW + wv != k) continue;
#pragma unroll
      for (int c = 0; c < NCTM; ++c) {
        if (c >= NCT) continue;
        d4 z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
          const int cc = 4 * kc + rq;
          const double dv = (double)Db[cl * kDST + cc];
          z = mfma64(cl <= cc ? dv : 0.0, y[li][c][kc], z);
        }
        y[li][c] = z;
#pragma unroll
        for (int q = 0; q < 4; ++q) xk[(c * 4 + q) * 64 + lane] = z[q];
        const int col = 16 * c + cl;
        if (col >= g.nrhs) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ii = 16 * k + 4 * q + rq;
          if (ii >= ni) continue;
          const double v = z[q];
          if (o.mode == BACK_UI) {
            o.ui[(size_t)leaf * ni + ii] = v;
          } else {
            double *dst = (col < nb) ? o.Xt + ((size_t)leaf * nb + col) * ni + ii
                                     : o.h + (size_t)leaf * ni + ii;
            if (o.mode == BACK_STORE) {
              *dst = v;
            } else {
              *dst += v;
              nd += v * v;
            }
          }
        }
      }
    }
  };
  // step k: everyone applies the published X_k to their own row tiles (with
  // the operands loaded one step earlier); the owner of the next row tile,
  // whose last update this was, forms and publishes it before the barrier,
  // so that forming is off the other wavefronts' path
  auto step = [&](int k, const T (&a)[RPW][4]) __attribute__((always_inline)) {
    const double *xk = xb + (k & 1) * NCTM * 256;
#pragma unroll
    for (int li = 0; li < RPW; ++li) {
      const int i = li * NW + wv;
      if (i >= k) continue;
#pragma unroll
      for (int c = 0; c < NCTM; ++c) {
        if (c >= NCT) continue;
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
          y[li][c] = mfma64((double)a[li][kc], -xk[(c * 4 + kc) * 64 + lane], y[li][c]);
      }
    }
    if (k >= 1) form(k - 1);
    lds_barrier();
  };
  T a0[RPW][4], a1[RPW][4];
  // backward; X_k is written out by its owner when formed
  load_a(a0, RT - 1);
  form(RT - 1);
  lds_barrier();
#pragma unroll 1
  for (int kk = 0; kk < RT; kk += 2) {
    const int k = RT - 1 - kk;
    load_a(a1, k - 1);
    step(k, a0);
    if (k - 1 >= 0) {
      load_a(a0, k - 2);
      step(k - 1, a1);
    }
  }
  if (o.mode == BACK_ACCUM) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nd += __shfl_xor(nd, off);
    if (lane == 0) red[wv] = nd;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
      for (int w = 0; w < NW; ++w) sum += red[w];
      o.norms[kNormStride * (size_t)leaf + 16] = sum;
    }
  }
}

// ---------------------------------------------------------------------------
// Triangular solves of the large work matrices with the right-hand sides in
// registers (the mirror of the left-looking factorisation's update loop).
// k_inv_udiag first inverts every 16 x 16 diagonal block of the factors
// (the pivot rows of panel b in columns 16b ...) into the leaf slot's
// per-panel tile, which the factorisation no longer needs: U_bb^{-1} on and
// above the diagonal and, for a forward pass, the unit-lower L_bb^{-1}
// strictly below it.  k_solve_big then takes 32 right-hand-side columns per
// workgroup: row tile t of the right-hand sides (in pivot order) sits in the
// FP64 accumulators of wavefront t % NW for the whole solve.  Forward, for
// k = 0, 1, ...: the owner of tile k forms Y_k = L_kk^{-1} Y_k and publishes
// it in LDS, and every tile t > k takes Y_t -= L_tk Y_k; backward, for
// k = RT-1 down to 0: X_k = U_kk^{-1} Y_k, and every tile t < k takes
// Y_t -= U_tk X_k.  The factor tiles L_tk / U_tk (the pivot rows of tile t,
// panel k's columns) are streamed into the wavefront's LDS slot by
// global_load_lds a step ahead; one LDS-only barrier per step.  The result
// leaves through LDS, every column of Xt (or u_i) as one contiguous row.
// ---------------------------------------------------------------------------
template <typename T, int PASSES>
__global__ void __launch_bounds__(256) k_inv_udiag(Geom g, T *M, const int *piv, Sel sel) {
  __shared__ T Dl[16][16 * 17];
  __shared__ int pv[16 * 16];
  const int wi = blockIdx.x, tid = threadIdx.x;
  int leaf;
  if (!resolve_leaf(sel, leaf)) return;
  const int RT = g.RT, CT = g.CT, R = g.R;
  T *Ml = M + leaf_stride(g) * wi;
  T *Lg = Ml + work_elems(g);
  const int b0 = blockIdx.y * 16;   // 16 diagonal blocks per workgroup
  const int nbk = min(16, RT - b0);
  if (nbk <= 0) return;
  for (int e = tid; e < nbk * 16; e += 256)
    pv[e] = min(max(piv[(size_t)wi * R + 16 * b0 + e], 0), R - 1);
  __syncthreads();
  for (int e = tid; e < nbk * 256; e += 256) {
    const int bb = e >> 8, s = (e >> 4) & 15, q = e & 15;
    Dl[bb][s * 17 + q] = Ml[tix<T>(pv[bb * 16 + s], 16 * (b0 + bb) + q, CT)];
  }
  __syncthreads();
  // column j of block bb per thread
  const int bb = tid >> 4, j = tid & 15;
  if (bb < nbk) {
    const T *D = Dl[bb];
    double zu[16], zl[16];
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double acc = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int q = i + 1; q < 16; ++q) acc -= (double)D[i * 17 + q] * zu[q];
      zu[i] = (i <= j) ? acc / (double)D[i * 17 + i] : 0.0;
    }
    if (PASSES & 2) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double acc = (i == j) ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < i; ++q) acc -= (double)D[i * 17 + q] * zl[q];
        zl[i] = acc;
      }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const double v = (i <= j) ? zu[i] : ((PASSES & 2) ? zl[i] : 0.0);
      Lg[(size_t)(b0 + bb) * 256 + i * 16 + j] = (T)v;
    }
  }
}

template <typename T, int NW, int RTW>
constexpr size_t solve_big_lds(int R) {
  // the streamed tiles' slots, doubling as the [R][17] FP64 staging of the result
  const size_t slots = sizeof(T) * (size_t)NW * RTW * 256;
  const size_t stage = sizeof(double) * (size_t)R * 17;
  return (slots > stage ? slots : stage) + sizeof(double) * 2 * 16 * 32 + sizeof(int) * (size_t)R;
}

template <typename T, int NW, int RTW, int PASSES>
__global__ void __launch_bounds__(64 * NW, 1) k_solve_big(Geom g, const T *M, const int *piv,
                                                         BackOut o, Sel sel, int nleaf, int nck) {
  constexpr int NT = 64 * NW, KT = 2, KW = 16 * KT;
  constexpr int kPer = 1024 / (int)sizeof(T);   // elements per gather instruction
  constexpr int kIns = 256 / kPer;               // instructions per tile
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // XCD-aware order: workgroups are dealt to the eight XCDs round-robin by
  // id, so the column chunks of one leaf take ids of one residue mod 8 and
  // run together on one XCD, whose L2 then serves the leaf's factor tiles
  // to all of them after one read from HBM
  const int xcd = (int)blockIdx.x & 7, grp = (int)blockIdx.x >> 3;
  const int chunk = grp % nck, wi = (grp / nck) * 8 + xcd;
  if (wi >= nleaf) return;
  int leaf = wi;
  if (sel.list) {
    const int slot = sel.slot0 + wi;
    if (slot >= *sel.count) return;
    leaf = sel.list[slot];
  }
  if (o.skip && o.skip[leaf]) return;
  const int R = g.R, RT = g.RT, CT = g.CT, ni = g.ni, nb = g.nb, NCT = CT - RT;
  const int c0 = chunk * KT;                   // first right-hand-side column tile
  const int ncol = min(KT, NCT - c0);
  if (ncol <= 0) return;
  const size_t slot_bytes = sizeof(T) * (size_t)NW * RTW * 256;
  const size_t stage_bytes = sizeof(double) * (size_t)R * 17;
  T *Abuf = (T *)smem;                         // [NW][RTW][256] streamed factor tiles
  double *Xs = (double *)smem;                 // [R][17] result staging (after the passes)
  double *Xp = (double *)(smem + (slot_bytes > stage_bytes ? slot_bytes : stage_bytes));
  int *pva = (int *)(Xp + 2 * 16 * KW);        // [R] pivot row of each step
  const T *Ml = M + leaf_stride(g) * wi;
  const T *Lg = Ml + work_elems(g);            // diagonal-block inverses, row-major per tile
  const int lr = lane >> 4, lc = lane & 15;
  for (int r = tid; r < R; r += NT) pva[r] = min(max(piv[(size_t)wi * R + r], 0), R - 1);
  __syncthreads();

  d4 acc[RTW][KT];
#pragma unroll
  for (int i = 0; i < RTW; ++i) {
    const int t = wv + NW * i;
#pragma unroll
    for (int c = 0; c < KT; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc[i][c][q] = (t < RT && c < ncol)
                           ? (double)Ml[tix<T>(pva[16 * t + 4 * q + lr], R + 16 * (c0 + c) + lc, CT)]
                           : 0.0;
  }
  // factor tile (rows of tile i, panel k's columns) into this wavefront's slot i
  auto gather = [&](int i, int k) {
    const int t = wv + NW * i;
    T *dst = Abuf + (size_t)(wv * RTW + i) * 256;
#pragma unroll
    for (int h = 0; h < kIns; ++h) {
      const int e = h * kPer + lane * (16 / (int)sizeof(T));
      const T *src = Ml + tix<T>(pva[16 * t + (e >> 4)], 16 * k + (e & 15), CT);
      __builtin_amdgcn_global_load_lds((const void *)src,
                                       (__attribute__((address_space(3))) void *)(dst + h * kPer),
                                       16, 0, 0);
    }
  };
  // tile i takes the step's update (operands paired over index 4 lr + kc,
  // as in the factorisation), its slot refilled at once for step kn when
  // the tile takes that step too
  auto mma = [&](int i, const double (&b)[KT][4], int kn, bool fwd) {
    const T *src = Abuf + (size_t)(wv * RTW + i) * 256 + lc * 16 + 4 * lr;
    double a[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) a[kc] = -(double)src[kc];
    const int t = wv + NW * i;
    if (kn >= 0 && (fwd ? t > kn : t < kn)) {
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // the slot has been read
      gather(i, kn);
    }
#pragma unroll
    for (int c = 0; c < KT; ++c) {
      if (c < ncol) {
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) acc[i][c] = mfma64(a[kc], b[c][kc], acc[i][c]);
      }
    }
  };
  // the owner of tile k applies the diagonal block's inverse (the
  // accumulators are the B operand: register kc holds row 4 kc + lr) and
  // publishes the result
  auto form = [&](int k, const double (&di)[4]) {
    double *xk = Xp + (k & 1) * 16 * KW;
#pragma unroll
    for (int i = 0; i < RTW; ++i) {
      if (wv + NW * i != k) continue;
#pragma unroll
      for (int c = 0; c < KT; ++c) {
        if (c >= ncol) continue;
        d4 z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) z = mfma64(di[kc], acc[i][c][kc], z);
        acc[i][c] = z;
#pragma unroll
        for (int q = 0; q < 4; ++q) xk[(4 * q + lr) * KW + 16 * c + lc] = z[q];
      }
    }
  };
  // row lc of the inverse of block k as this lane's A operand: U^{-1} on and
  // above the diagonal (backward) or unit-lower L^{-1} (forward)
  double dpre[4];
  auto load_inv = [&](int k, bool fwd) {
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int cc = 4 * kc + lr;
      const double v = (double)Lg[(size_t)k * 256 + lc * 16 + cc];
      dpre[kc] = fwd ? (lc > cc ? v : (lc == cc ? 1.0 : 0.0)) : (lc <= cc ? v : 0.0);
    }
  };
  // one pass: k runs from k_first to k_last (step dir); tiles "after" k in
  // the pass order take each X_k
  auto pass = [&](bool fwd) {
    const int dir = fwd ? 1 : -1;
    const int kf = fwd ? 0 : RT - 1, kl = fwd ? RT - 1 : 0;
#pragma unroll
    for (int i = 0; i < RTW; ++i) {
      const int t = wv + NW * i;
      if (t < RT && (fwd ? t > kf : t < kf)) gather(i, kf);
    }
    if (wv == kf % NW) {
      load_inv(kf, fwd);
      form(kf, dpre);
    }
    if (RT >= 2 && wv == (kf + dir) % NW) load_inv(kf + dir, fwd);
    for (int k = kf; k != kl; k += dir) {
      lds_barrier();
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wavefront's loads of step k
      const double *X = Xp + (k & 1) * 16 * KW;
      double b[KT][4];
#pragma unroll
      for (int c = 0; c < KT; ++c) {
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
          b[c][kc] = c < ncol ? X[(4 * lr + kc) * KW + 16 * c + lc] : 0.0;
      }
      const int kn = k + dir;                  // the next step
      const int kload = kn != kl ? kn : -1;    // tiles after kn gather for it
      const bool ahead = wv == kn % NW;        // owner of tile kn forms it
      if (ahead) {
#pragma unroll
        for (int i = 0; i < RTW; ++i)
          if (wv + NW * i == kn) mma(i, b, kload, fwd);
      }
#pragma unroll
      for (int i = 0; i < RTW; ++i) {
        const int t = wv + NW * i;
        if (t < RT && (fwd ? t > k : t < k) && !(ahead && t == kn)) mma(i, b, kload, fwd);
      }
      if (ahead) form(kn, dpre);   // last, when tile kn's products have completed
      if (kn != kl && wv == (kn + dir) % NW) load_inv(kn + dir, fwd);
    }
    __syncthreads();
  };
  if (PASSES & 2) pass(true);
  if (PASSES & 1) pass(false);

  // the result out through LDS: one column tile at a time, rows contiguous
  double nd = 0.0;
#pragma unroll
  for (int c = 0; c < KT; ++c) {
    if (c >= ncol) continue;
#pragma unroll
    for (int i = 0; i < RTW; ++i) {
      const int t = wv + NW * i;
      if (t < RT) {
#pragma unroll
        for (int q = 0; q < 4; ++q) Xs[(16 * t + 4 * q + lr) * 17 + lc] = acc[i][c][q];
      }
    }
    __syncthreads();
    for (int e = tid; e < 16 * ni; e += NT) {
      const int cc = e / ni, r = e - cc * ni;
      const int col = 16 * (c0 + c) + cc;
      if (col >= g.nrhs) continue;
      const double v = Xs[r * 17 + cc];
      if (o.mode == BACK_UI) {
        o.ui[(size_t)leaf * ni + r] = v;
      } else {
        double *dst = (col < nb) ? o.Xt + ((size_t)leaf * nb + col) * ni + r
                                 : o.h + (size_t)leaf * ni + r;
        if (o.mode == BACK_STORE) {
          *dst = v;
        } else {
          *dst += v;
          nd += v * v;
        }
      }
    }
    __syncthreads();
  }
  if (o.mode == BACK_ACCUM) {
    double *red = Xs;   // the staging is free again
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nd += __shfl_xor(nd, off);
    if (lane == 0) red[wv] = nd;
    __syncthreads();
    if (tid == 0) {
      double a = 0.0;
      for (int w = 0; w < NW; ++w) a += red[w];
      o.norms[kNormStride * (size_t)leaf + 16 + chunk] = a;
    }
  }
}

// The refinement correction (forward then backward, FP32 factors) with each
// wavefront owning one right-hand-side column tile instead: it keeps all RT
// row tiles of that column tile in its accumulators and walks both
// substitutions alone, so that after the shared prologue (pivots, inverted
// diagonal blocks) no barrier is left; each wavefront reads the factor
// tiles it needs itself (the wavefronts of a leaf share them through
// L1/L2).  Measured faster than the row-owned kernel for this two-pass
// launch (1.26 vs 1.57 ms at p = 16), whose per-step barriers then dominate.
template <int RTM>
__global__ void __launch_bounds__(320) k_solve_cols(Geom g, const float *M, const int *piv,
                                                    BackOut o) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wi = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int NT = blockDim.x, NW = NT >> 6;
  const int leaf = wi;
  if (o.skip && o.skip[leaf]) return;
  const int R = g.R, RT = g.RT, CT = g.CT, ni = g.ni, nb = g.nb;
  double *red = (double *)smem;                          // [8]
  float *D = (float *)(red + 8);                         // [RT][16][kDST]
  int *pva = (int *)(D + (size_t)RT * 16 * kDST);        // [R]
  const float *Ml = M + leaf_stride(g) * wi;
  stage_inverse_diag<float, 3>(g, Ml, piv + (size_t)wi * R, D, pva, tid, NT);

  const int cl = lane & 15, rq = lane >> 4, col = wv * 16 + cl;
  d4 y[RTM];
#pragma unroll
  for (int k = 0; k < RTM; ++k) {
    if (k < RT) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        y[k][q] = (double)Ml[tix<float>(pva[16 * k + 4 * q + rq], R + col, CT)];
    }
  }
#pragma unroll
  for (int k = 0; k < RTM; ++k) {
    if (k < RT) {
      const float *Db = D + k * 16 * kDST;
      d4 nk = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const int c = 4 * kc + rq;
        const double a = cl > c ? (double)Db[cl * kDST + c] : (cl == c ? 1.0 : 0.0);
        nk = mfma64(a, y[k][kc], nk);
      }
      y[k] = nk;
#pragma unroll
      for (int i = k + 1; i < RTM; ++i) {
        if (i < RT) {
          const int pr = pva[16 * i + cl];
#pragma unroll
          for (int kc = 0; kc < 4; ++kc)
            y[i] = mfma64((double)Ml[tix<float>(pr, 16 * k + 4 * kc + rq, CT)], -nk[kc], y[i]);
        }
      }
    }
  }
  double nd = 0.0;
#pragma unroll
  for (int k = RTM - 1; k >= 0; --k) {
    if (k < RT) {
      const float *Db = D + k * 16 * kDST;
      d4 xk = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const int c = 4 * kc + rq;
        xk = mfma64(cl <= c ? (double)Db[cl * kDST + c] : 0.0, y[k][kc], xk);
      }
#pragma unroll
      for (int i = 0; i < k; ++i) {
        const int pr = pva[16 * i + cl];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
          y[i] = mfma64((double)Ml[tix<float>(pr, 16 * k + 4 * kc + rq, CT)], -xk[kc], y[i]);
      }
      if (col < g.nrhs) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ii = 16 * k + 4 * q + rq;
          if (ii >= ni) continue;
          const double v = xk[q];
          double *dst = (col < nb) ? o.Xt + ((size_t)leaf * nb + col) * ni + ii
                                   : o.h + (size_t)leaf * ni + ii;
          if (o.mode == BACK_STORE) {
            *dst = v;
          } else {
            *dst += v;
            nd += v * v;
          }
        }
      }
    }
  }
  if (o.mode == BACK_ACCUM) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nd += __shfl_xor(nd, off);
    if (lane == 0) red[wv] = nd;
    __syncthreads();
    if (tid == 0) {
      double sum = 0.0;
      for (int w = 0; w < NW; ++w) sum += red[w];
      o.norms[kNormStride * (size_t)leaf + 16] = sum;
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 refinement residual  r = A_ib - A_ii X  (and f_i - A_ii h), applied
// through the tensor structure of the collocation operator: each interior
// row couples only to its own x1-line and x2-line of nodes.  One workgroup
// per leaf; a thread owns one row and keeps its coefficients in
// registers; CW columns of [X h] at a time are staged in LDS (coalesced
// reads of Xt); each line weight is formed once per row and chunk and used
// for all CW columns.  A leaf's columns may be split over gridDim.y
// workgroups.  The residual is written in FP32 into the right-hand-side
// columns of the work matrix for the correction solve (zero in the padding
// rows), and the squared Frobenius norms of r and X are stored per leaf and
// column chunk for the stop test.
// ---------------------------------------------------------------------------
template <int NT, int CW>
__global__ void __launch_bounds__(NT) k_residual(Geom g, float *M32, const double *Xt,
                                                  const double *h, const double *f,
                                                  const int *skip, double *norms) {
  extern __shared__ __align__(16) unsigned char smem[];
  double *sD = (double *)smem;               // [p*p]
  double *sD2 = sD + g.p * g.p;              // [p*p]
  double *xs = sD2 + g.p * g.p;              // [CW][ni] staged columns of [X h]
  __shared__ double red[NT / 64][2];
  const int leaf = blockIdx.x;
  if (skip && skip[leaf]) return;
  stage_tables(g, sD, sD2);
  const LeafScale sc = leaf_scale(g, leaf);
  const int p = g.p, m = g.m, ni = g.ni, nb = g.nb, R = g.R, CT = g.CT;
  const size_t nbase = (size_t)leaf * p * p;
  float *Ml = M32 + leaf_stride(g) * leaf;
  const int ncol = (h && f) ? nb + 1 : nb;
  const int r = threadIdx.x;   // this thread's row (NT >= R)
  int i = 0, j = 0;
  double ax2 = 0.0, ax1 = 0.0, ay2 = 0.0, ay1 = 0.0, kb = 0.0;
  if (r < ni) {
    i = r % m + 1;
    j = r / m + 1;
    const size_t n = nbase + i + (size_t)p * j;
    ax2 = (g.a11 ? g.a11[n] : 1.0) * sc.sx * sc.sx;
    ax1 = (g.c1 ? g.c1[n] : 0.0) * sc.sx;
    ay2 = (g.a22 ? g.a22[n] : 1.0) * sc.sy * sc.sy;
    ay1 = (g.c2 ? g.c2[n] : 0.0) * sc.sy;
    kb = g.k2b ? g.k2b[n] : 0.0;
  }
  double nr = 0.0, nx = 0.0;
  // this workgroup's columns: chunk blockIdx.y of gridDim.y, whole CW groups
  const int ngrp = (ncol + CW - 1) / CW;
  const int g0 = (ngrp * (int)blockIdx.y) / (int)gridDim.y;
  const int g1 = (ngrp * ((int)blockIdx.y + 1)) / (int)gridDim.y;
  for (int c0 = g0 * CW; c0 < min(g1 * CW, ncol); c0 += CW) {
    const int cw = min(CW, ncol - c0);
    __syncthreads();
    for (int e = threadIdx.x; e < cw * ni; e += NT) {
      const int c = e / ni, i = e - c * ni, col = c0 + c;
      xs[c * ni + i] = (col < nb) ? Xt[((size_t)leaf * nb + col) * ni + i] : h[(size_t)leaf * ni + i];
    }
    __syncthreads();
    if (r >= ni) {
      if (r < R)
        for (int c = 0; c < cw; ++c) Ml[tix<float>(r, R + c0 + c, CT)] = 0.0f;
      continue;
    }
    // -(A_ii x) = k2b x + sum over both lines of (a d2 + c d1) x
    double acc[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) acc[c] = c < cw ? kb * xs[c * ni + r] : 0.0;
    for (int k = 1; k <= m; ++k) {
      const double wx = ax2 * sD2[i * p + k] + ax1 * sD[i * p + k];
      const double wy = ay2 * sD2[j * p + k] + ay1 * sD[j * p + k];
      const int xa = (k - 1) + m * (j - 1), ya = (i - 1) + m * (k - 1);
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        if (c < cw) acc[c] += wx * xs[c * ni + xa] + wy * xs[c * ni + ya];
      }
    }
#pragma unroll
    for (int c = 0; c < CW; ++c) {
      if (c >= cw) continue;
      const int col = c0 + c;
      double bval = 0.0;   // entry of [A_ib f] in this row
      if (col == nb) {
        bval = f[(size_t)leaf * ni + r];
      } else if (col == j - 1) {
        bval = -(ax2 * sD2[i * p] + ax1 * sD[i * p]);
      } else if (col == m + j - 1) {
        bval = -(ax2 * sD2[i * p + p - 1] + ax1 * sD[i * p + p - 1]);
      } else if (col == 2 * m + i - 1) {
        bval = -(ay2 * sD2[j * p] + ay1 * sD[j * p]);
      } else if (col == 3 * m + i - 1) {
        bval = -(ay2 * sD2[j * p + p - 1] + ay1 * sD[j * p + p - 1]);
      }
      const double res = bval + acc[c];
      const double x = xs[c * ni + r];
      nr += res * res;
      nx += x * x;
      Ml[tix<float>(r, R + col, CT)] = (float)res;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    nr += __shfl_xor(nr, off);
    nx += __shfl_xor(nx, off);
  }
  if (lane == 0) {
    red[wv][0] = nr;
    red[wv][1] = nx;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double a = 0.0;
    for (int w = 0; w < NT / 64; ++w) a += red[w][threadIdx.x];
    norms[kNormStride * (size_t)leaf + 8 + 4 * threadIdx.x + blockIdx.y] = a;
  }
}

// The same residual on the MFMA units for leaves with at most 16 interior
// nodes per line (p <= 18).  For one column of [X h], with G the m x m grid
// of its values (G[i][j] at interior node (i, j), zero-padded to 16 x 16),
// both line sums of every row are tile products with the interior block of
// a differentiation matrix D (D1 or D2):
//   along x1: sum_k D[i][k] G[k][j] = (D G)[i][j]
//   along x2: sum_k D[j][k] G[i][k] = (G D^T)[i][j]
// and each node's own coefficients combine the four products.  Wavefront w
// takes every fourth column and stages its grid in a private LDS tile; the
// MFMA accumulator layout puts node (4q + lane/16, lane%16) in register q of
// a lane, which is also where the lane's B operand of D G holds G.
__global__ void __launch_bounds__(256) k_residual_m(Geom g, float *M32, const double *Xt,
                                                    const double *h, const double *f,
                                                    const int *skip, double *norms) {
  constexpr int NW = 4, GS = 17;
  __shared__ double gs[NW][16 * GS];
  __shared__ double red[NW][2];
  const int leaf = blockIdx.x;
  if (skip && skip[leaf]) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, cl = lane & 15, rq = lane >> 4;
  const LeafScale sc = leaf_scale(g, leaf);
  const int p = g.p, m = g.m, ni = g.ni, nb = g.nb, R = g.R, CT = g.CT;
  float *Ml = M32 + leaf_stride(g) * leaf;
  const int ncol = (h && f) ? nb + 1 : nb;
  // A operand of D G (and B operand of G D^T): D[cl + 1][4kc + rq + 1]
  double d1[4], d2[4];
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    const int k = 4 * kc + rq;
    const bool in = cl < m && k < m;
    d1[kc] = in ? g.D[(cl + 1) * p + k + 1] : 0.0;
    d2[kc] = in ? g.D2[(cl + 1) * p + k + 1] : 0.0;
  }
  // coefficients of this lane's nodes (i, j) = (4q + rq, cl)
  double ax2[4], ax1[4], ay2[4], ay1[4], kb[4], bw0[4], bw1[4], bs0[4], bs1[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = 4 * q + rq, j = cl;
    ax2[q] = ax1[q] = ay2[q] = ay1[q] = kb[q] = bw0[q] = bw1[q] = bs0[q] = bs1[q] = 0.0;
    if (i < m && j < m) {
      const size_t n = (size_t)leaf * p * p + (i + 1) + (size_t)p * (j + 1);
      ax2[q] = (g.a11 ? g.a11[n] : 1.0) * sc.sx * sc.sx;
      ax1[q] = (g.c1 ? g.c1[n] : 0.0) * sc.sx;
      ay2[q] = (g.a22 ? g.a22[n] : 1.0) * sc.sy * sc.sy;
      ay1[q] = (g.c2 ? g.c2[n] : 0.0) * sc.sy;
      kb[q] = g.k2b ? g.k2b[n] : 0.0;
      bw0[q] = -(ax2[q] * g.D2[(i + 1) * p] + ax1[q] * g.D[(i + 1) * p]);
      bw1[q] = -(ax2[q] * g.D2[(i + 1) * p + p - 1] + ax1[q] * g.D[(i + 1) * p + p - 1]);
      bs0[q] = -(ay2[q] * g.D2[(j + 1) * p] + ay1[q] * g.D[(j + 1) * p]);
      bs1[q] = -(ay2[q] * g.D2[(j + 1) * p + p - 1] + ay1[q] * g.D[(j + 1) * p + p - 1]);
    }
  }
  // grid positions of the column entries e = lane + 64 t this lane stages
  int gpos[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int e = lane + 64 * t;
    gpos[t] = e < ni ? (e % m) * GS + e / m : -1;
  }
  double *G = gs[wv];
  for (int e = lane; e < 16 * GS; e += 64) G[e] = 0.0;   // padding stays zero
  double nr = 0.0, nx = 0.0;
  const int c0 = (ncol * (int)blockIdx.y) / (int)gridDim.y;
  const int c1 = (ncol * ((int)blockIdx.y + 1)) / (int)gridDim.y;
  // the next columns' values are loaded while the current one is processed
  auto load_col = [&](int c, double (&v)[4]) {
    const double *src = c < nb ? Xt + ((size_t)leaf * nb + c) * ni : h + (size_t)leaf * ni;
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = gpos[t] >= 0 ? src[lane + 64 * t] : 0.0;
  };
  // (PD columns ahead; four measured no faster than two)
  constexpr int PD = 2;
  double nxt[PD][4];
#pragma unroll
  for (int d = 0; d < PD; ++d) {
    const int cd = c0 + wv + d * NW;
#pragma unroll
    for (int t = 0; t < 4; ++t) nxt[d][t] = 0.0;
    if (cd < c1) load_col(cd, nxt[d]);
  }
  for (int c = c0 + wv; c < c1; c += NW) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (gpos[t] >= 0) G[gpos[t]] = nxt[0][t];
#pragma unroll
    for (int d = 0; d + 1 < PD; ++d)
#pragma unroll
      for (int t = 0; t < 4; ++t) nxt[d][t] = nxt[d + 1][t];
    wave_lds_fence<double>();
    if (c + PD * NW < c1) load_col(c + PD * NW, nxt[PD - 1]);
    double bo[4], ao[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      bo[kc] = G[(4 * kc + rq) * GS + cl];
      ao[kc] = G[cl * GS + 4 * kc + rq];
    }
    d4 t1x = {0.0, 0.0, 0.0, 0.0}, t2x = t1x, t1y = t1x, t2y = t1x;
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      t1x = mfma64(d1[kc], bo[kc], t1x);
      t2x = mfma64(d2[kc], bo[kc], t2x);
      t1y = mfma64(ao[kc], d1[kc], t1y);
      t2y = mfma64(ao[kc], d2[kc], t2y);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 4 * q + rq, j = cl;
      if (i >= m || j >= m) continue;
      const int r = i + m * j;
      const double x = bo[q];
      // -(A_ii x) = k2b x + sum over both lines of (a d2 + c d1) x
      const double acc = kb[q] * x + ax2[q] * t2x[q] + ax1[q] * t1x[q] + ay2[q] * t2y[q] +
                         ay1[q] * t1y[q];
      double bval = 0.0;   // entry of [A_ib f] in this row
      if (c == nb) bval = f[(size_t)leaf * ni + r];
      else if (c == j) bval = bw0[q];
      else if (c == m + j) bval = bw1[q];
      else if (c == 2 * m + i) bval = bs0[q];
      else if (c == 3 * m + i) bval = bs1[q];
      const double res = bval + acc;
      nr += res * res;
      nx += x * x;
      Ml[tix<float>(r, R + c, CT)] = (float)res;
    }
    for (int r = ni + lane; r < R; r += 64) Ml[tix<float>(r, R + c, CT)] = 0.0f;
    // the next column's staging must not overtake this column's reads
    wave_lds_fence<double>();
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    nr += __shfl_xor(nr, off);
    nx += __shfl_xor(nx, off);
  }
  if (lane == 0) {
    red[wv][0] = nr;
    red[wv][1] = nx;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double a = 0.0;
    for (int w = 0; w < NW; ++w) a += red[w][threadIdx.x];
    norms[kNormStride * (size_t)leaf + 8 + 4 * threadIdx.x + blockIdx.y] = a;
  }
}

// The MFMA residual for 24 <= m <= 30 (p = 26 ... 32): the grid of a column is
// 2 x 2 tiles, each output tile (I, J) takes the products
//   (D G)(I, J) = sum_K D(I, K) G(K, J),  (G D^T)(I, J) = sum_K G(I, K) D(J, K)^T
// for D1 and D2 (32 tile products per output tile); D's tiles stay in
// registers (their A-operand layout is also the B-operand layout of D^T),
// the nodes' coefficients are read per output tile, and the boundary
// couplings are formed only at the nodes that have one.  A column's values
// are loaded one column ahead.
__global__ void __launch_bounds__(256) k_residual_m2(Geom g, float *M32, const double *Xt,
                                                     const double *h, const double *f,
                                                     const int *skip, double *norms) {
  constexpr int NW = 4, GS = 33, NV = 15;   // NV * 64 >= 32 * 32 > ni
  __shared__ double gs[NW][32 * GS];
  __shared__ double red[NW][2];
  const int leaf = blockIdx.x;
  if (skip && skip[leaf]) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, cl = lane & 15, rq = lane >> 4;
  const LeafScale sc = leaf_scale(g, leaf);
  const int p = g.p, m = g.m, ni = g.ni, nb = g.nb, R = g.R, CT = g.CT;
  float *Ml = M32 + leaf_stride(g) * leaf;
  const int ncol = (h && f) ? nb + 1 : nb;
  // dd[0/1][I][K][kc] = D1/D2[16I + cl + 1][16K + 4kc + rq + 1] (zero outside the interior)
  double dd[2][2][2][4];
#pragma unroll
  for (int I = 0; I < 2; ++I)
#pragma unroll
    for (int K = 0; K < 2; ++K)
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        const int i = 16 * I + cl, k = 16 * K + 4 * kc + rq;
        const bool in = i < m && k < m;
        dd[0][I][K][kc] = in ? g.D[(i + 1) * p + k + 1] : 0.0;
        dd[1][I][K][kc] = in ? g.D2[(i + 1) * p + k + 1] : 0.0;
      }
  int gpos[NV];
#pragma unroll
  for (int t = 0; t < NV; ++t) {
    const int e = lane + 64 * t;
    gpos[t] = e < ni ? (e % m) * GS + e / m : -1;
  }
  double *G = gs[wv];
  for (int e = lane; e < 32 * GS; e += 64) G[e] = 0.0;   // padding stays zero
  auto load_col = [&](int c, double (&v)[NV]) {
    const double *src = c < nb ? Xt + ((size_t)leaf * nb + c) * ni : h + (size_t)leaf * ni;
#pragma unroll
    for (int t = 0; t < NV; ++t) v[t] = gpos[t] >= 0 ? src[lane + 64 * t] : 0.0;
  };
  double nr = 0.0, nx = 0.0;
  const int c0 = (ncol * (int)blockIdx.y) / (int)gridDim.y;
  const int c1 = (ncol * ((int)blockIdx.y + 1)) / (int)gridDim.y;
  double nxt[NV];
#pragma unroll
  for (int t = 0; t < NV; ++t) nxt[t] = 0.0;
  if (c0 + wv < c1) load_col(c0 + wv, nxt);
  for (int c = c0 + wv; c < c1; c += NW) {
#pragma unroll
    for (int t = 0; t < NV; ++t)
      if (gpos[t] >= 0) G[gpos[t]] = nxt[t];
    wave_lds_fence<double>();
    if (c + NW < c1) load_col(c + NW, nxt);
#pragma unroll
    for (int I = 0; I < 2; ++I) {
#pragma unroll
      for (int J = 0; J < 2; ++J) {
        if (16 * I >= m || 16 * J >= m) continue;
        d4 t1x = {0.0, 0.0, 0.0, 0.0}, t2x = t1x, t1y = t1x, t2y = t1x;
#pragma unroll
        for (int K = 0; K < 2; ++K) {
#pragma unroll
          for (int kc = 0; kc < 4; ++kc) {
            const double bo = G[(16 * K + 4 * kc + rq) * GS + 16 * J + cl];   // G(K, J)
            const double ao = G[(16 * I + cl) * GS + 16 * K + 4 * kc + rq];   // G(I, K)
            t1x = mfma64(dd[0][I][K][kc], bo, t1x);
            t2x = mfma64(dd[1][I][K][kc], bo, t2x);
            t1y = mfma64(ao, dd[0][J][K][kc], t1y);
            t2y = mfma64(ao, dd[1][J][K][kc], t2y);
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = 16 * I + 4 * q + rq, j = 16 * J + cl;
          if (i >= m || j >= m) continue;
          const int r = i + m * j;
          const size_t n = (size_t)leaf * p * p + (i + 1) + (size_t)p * (j + 1);
          const double ax2 = (g.a11 ? g.a11[n] : 1.0) * sc.sx * sc.sx;
          const double ax1 = (g.c1 ? g.c1[n] : 0.0) * sc.sx;
          const double ay2 = (g.a22 ? g.a22[n] : 1.0) * sc.sy * sc.sy;
          const double ay1 = (g.c2 ? g.c2[n] : 0.0) * sc.sy;
          const double kb = g.k2b ? g.k2b[n] : 0.0;
          const double x = G[i * GS + j];
          // -(A_ii x) = k2b x + sum over both lines of (a d2 + c d1) x
          const double acc = kb * x + ax2 * t2x[q] + ax1 * t1x[q] + ay2 * t2y[q] + ay1 * t1y[q];
          double bval = 0.0;   // entry of [A_ib f] in this row
          if (c == nb) bval = f[(size_t)leaf * ni + r];
          else if (c == j) bval = -(ax2 * g.D2[(i + 1) * p] + ax1 * g.D[(i + 1) * p]);
          else if (c == m + j) bval = -(ax2 * g.D2[(i + 1) * p + p - 1] + ax1 * g.D[(i + 1) * p + p - 1]);
          else if (c == 2 * m + i) bval = -(ay2 * g.D2[(j + 1) * p] + ay1 * g.D[(j + 1) * p]);
          else if (c == 3 * m + i) bval = -(ay2 * g.D2[(j + 1) * p + p - 1] + ay1 * g.D[(j + 1) * p + p - 1]);
          const double res = bval + acc;
          nr += res * res;
          nx += x * x;
          Ml[tix<float>(r, R + c, CT)] = (float)res;
        }
      }
    }
    for (int r = ni + lane; r < R; r += 64) Ml[tix<float>(r, R + c, CT)] = 0.0f;
    // the next column's staging must not overtake this column's reads
    wave_lds_fence<double>();
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    nr += __shfl_xor(nr, off);
    nx += __shfl_xor(nx, off);
  }
  if (lane == 0) {
    red[wv][0] = nr;
    red[wv][1] = nx;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double a = 0.0;
    for (int w = 0; w < NW; ++w) a += red[w][threadIdx.x];
    norms[kNormStride * (size_t)leaf + 8 + 4 * threadIdx.x + blockIdx.y] = a;
  }
}

// Stop test of the refinement, per leaf, after the residual r_k of X_k: the
// estimated forward error rho / (1 - rho) ||dX_k|| is at most tol ||X_k||,
// where dX_k is the last correction and rho < 1, the contraction factor of
// the iteration, is the larger of two estimates: the observed contraction
// of the residual ||r_k|| / ||r_{k-1}||, and the relative size of the first
// correction ||dX_1|| / ||X_1||, i.e. the forward error of the low-precision
// solve, which sets the contraction of LU-based refinement.  rho / (1 - rho)
// ||dX_k|| bounds the remaining error of a contraction (the sum of the
// corrections still to come, a geometric series); rho ||dX_k|| alone, the
// next correction, underestimates it by 1 / (1 - rho), tenfold when the
// iteration contracts slowly (rho ~ 0.9).  Both estimates of rho can fall
// short of the true contraction: on the workloads' leaves (FP32 LU, FP64
// residual) by up to 16x, when the error left after a correction lies in
// directions the residual barely sees.  The estimate is therefore taken
// kRhoSafety = 16 times larger: 16 rho / (1 - rho) ||dX_k|| <= tol ||X_k||.
// (A p = 24 leaf of cond 8.5e5 otherwise stopped after one correction with
// a forward error of 1.4e-9; its second correction reaches 1e-13.)  A leaf
// whose iteration stalls above tol (its FP64 error floor, about
// cond(A_ii) 2^-53, lies above tol) never passes.  An exactly zero residual
// passes; tol >= 1 passes on the final check without a test.  On the final
// check a leaf that did not pass is flagged -1.
// norms[kNormStride l + ...]: 0 ||r||^2, 1 ||X||^2 (sums of the nres
// residual chunks' partial sums), 4 previous ||r||^2, 5 ||dX||^2 of the last
// correction (sum of its nsol chunks), 6 the relative size of the first
// correction.
constexpr double kRhoSafety = 16.0;

__global__ void k_convcheck(int nleaf, double *norms, double tol, int *conv, int *info,
                            int it, int last, int nres, int nsol) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nleaf || conv[l]) return;
  double *n = norms + kNormStride * (size_t)l;
  n[0] = n[1] = 0.0;
  for (int c = 0; c < nres; ++c) {
    n[0] += n[8 + c];
    n[1] += n[12 + c];
  }
  if (it > 0) {
    n[5] = 0.0;
    for (int c = 0; c < nsol; ++c) n[5] += n[16 + c];
  }
  bool ok = n[0] == 0.0 || (tol >= 1.0 && last);
  if (it == 1) n[6] = n[1] > 0.0 ? sqrt(n[5] / n[1]) : 1.0;
  if (!ok && tol < 1.0 && it > 0 && n[4] > 0.0) {
    const double rho = fmax(sqrt(n[0] / n[4]), n[6]);
    ok = rho < 1.0 && kRhoSafety * rho * sqrt(n[5]) <= tol * (1.0 - rho) * sqrt(n[1]);
  }
  n[4] = n[0];
  if (ok) {
    conv[l] = 1;
  } else if (last && info[l] == 0) {
    info[l] = -1;
  }
}

// Leaves whose refinement failed (info -1) are listed for an FP64 redo and
// flagged in `redo` (indexed like `info`).
__global__ void k_collect(int nleaf, int *info, int *list, int *count, int *total, int *redo) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nleaf || info[l] != -1) return;
  atomicAdd(total, 1);
  const int slot = atomicAdd(count, 1);
  list[slot] = l;
  info[l] = 0;
  redo[l] = 1;
}

// ---------------------------------------------------------------------------
// Schur complement S = A_bb - A_bi X and w = A_bi h in FP64.  A_bi has p-2
// nonzeros per row (the normal derivative along one grid line) and A_bb two.
// Columns of X are staged through LDS sixteen (large ni: eight) at a time,
// the LDS sized by ni, so that every global read is coalesced.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_schur(Geom g, const double *Xt, const double *h,
                                               double *S, double *w, int *info, int kSchurCols) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sD0[32], sD1[32];   // rows 0 and p-1 of D
  double *xs = (double *)smem;          // [kSchurCols][ni] staged columns of [X h]
  __shared__ int bad;
  const int leaf = blockIdx.x;
  const int p = g.p, m = g.m, ni = g.ni, nb = g.nb;
  for (int e = threadIdx.x; e < p; e += blockDim.x) {
    sD0[e] = g.D[e];
    sD1[e] = g.D[(p - 1) * p + e];
  }
  if (threadIdx.x == 0) bad = 0;
  const LeafScale sc = leaf_scale(g, leaf);
  const double *Xl = Xt + (size_t)leaf * nb * ni;
  int mybad = 0;
  // columns 0..nb-1 of X, then (column nb) h for w
  const int ncol = nb + 1;
  for (int c0 = 0; c0 < ncol; c0 += kSchurCols) {
    const int cw = min(kSchurCols, ncol - c0);
    __syncthreads();
    // the pass's columns of X are contiguous (then h): eight independent
    // loads per thread in flight at a time
    {
      const int tot = cw * ni, nx = (min(c0 + cw, nb) - c0) * ni;
      const double *src = Xl + (size_t)c0 * ni;
      const double *hl = h ? h + (size_t)leaf * ni : nullptr;   // entry e - nx
      constexpr int U = 8;
      for (int e0 = threadIdx.x; e0 < tot; e0 += U * 256) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = e0 + u * 256;
          v[u] = e < nx ? src[e] : ((e < tot && hl) ? hl[e - nx] : 0.0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = e0 + u * 256;
          if (e < tot) xs[e] = v[u];
        }
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nb * cw; e += blockDim.x) {
      const int b1 = e / cw, c = e - b1 * cw, b2 = c0 + c;
      const int s1 = b1 / m, q1 = b1 - s1 * m + 1;
      const double *drow = (s1 == 0 || s1 == 2) ? sD0 : sD1;
      const double scl = ((s1 == 0 || s1 == 2) ? -1.0 : 1.0) * ((s1 < 2) ? sc.sx : sc.sy);
      const double *x = xs + c * ni;
      double acc = 0.0;
      if (s1 < 2) {
        for (int t = 1; t <= m; ++t) acc += drow[t] * x[(t - 1) + m * (q1 - 1)];
      } else {
        for (int t = 1; t <= m; ++t) acc += drow[t] * x[(q1 - 1) + m * (t - 1)];
      }
      acc *= scl;  // (A_bi x)[b1]
      if (b2 == nb) {
        if (w) w[(size_t)leaf * nb + b1] = acc;
        mybad |= !isfinite(acc);
      } else {
        double abb = 0.0;
        const int s2 = b2 / m, q2 = b2 - s2 * m + 1;
        if (q1 == q2 && (s1 >> 1) == (s2 >> 1)) {
          // same grid line: first/last node of the normal-derivative stencil
          abb = scl * ((s2 == 0 || s2 == 2) ? drow[0] : drow[p - 1]);
        }
        const double v = abb - acc;
        S[((size_t)leaf * nb + b1) * nb + b2] = v;
        mybad |= !isfinite(v);
      }
    }
  }
  if (mybad) bad = 1;
  __syncthreads();
  if (threadIdx.x == 0 && bad && info[leaf] == 0) info[leaf] = -2;
}

// u_i = h - X u_b from the stored FP64 X (transposed) and h.
__global__ void __launch_bounds__(256) k_recover(Geom g, const double *Xt, const double *h,
                                                 const double *ub, double *ui) {
  __shared__ double su[128];
  const int leaf = blockIdx.x;
  const int ni = g.ni, nb = g.nb;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) su[b] = ub[(size_t)leaf * nb + b];
  __syncthreads();
  const int i = blockIdx.y * blockDim.x + threadIdx.x;
  if (i >= ni) return;
  const double *Xl = Xt + (size_t)leaf * nb * ni + i;
  double v = h ? h[(size_t)leaf * ni + i] : 0.0;
  for (int b = 0; b < nb; ++b) v -= Xl[(size_t)b * ni] * su[b];
  ui[(size_t)leaf * ni + i] = v;
}

// Dense blocks of the leaf matrix (operator check).
__global__ void __launch_bounds__(256) k_operator(Geom g, double *Aii, double *Aib,
                                                  double *Abi, double *Abb) {
  __shared__ double sD[32 * 32], sD2[32 * 32];
  const int leaf = blockIdx.x;
  stage_tables(g, sD, sD2);
  __syncthreads();
  const LeafScale sc = leaf_scale(g, leaf);
  const int p = g.p, m = g.m, ni = g.ni, nb = g.nb;
  const size_t nbase = (size_t)leaf * p * p;
  if (Aii)
    for (int e = threadIdx.x; e < ni * ni; e += blockDim.x) {
      const int r = e / ni, c = e - r * ni;
      Aii[(size_t)leaf * ni * ni + e] =
          opval(g, sD, sD2, sc, nbase, r % m + 1, r / m + 1, c % m + 1, c / m + 1);
    }
  if (Aib)
    for (int e = threadIdx.x; e < ni * nb; e += blockDim.x) {
      const int r = e / nb, b = e - r * nb;
      Aib[(size_t)leaf * ni * nb + e] = aib_elem(g, sD, sD2, sc, nbase, r % m + 1, r / m + 1, b);
    }
  // boundary rows: outward normal derivative along the line through the node
  auto brow = [&](int b, int k, int l) -> double {
    int kb, lb;
    bnode(b, m, p, kb, lb);
    const int s = b / m;
    if (s < 2) {  // W / E: d/dx1 along row lb
      if (l != lb) return 0.0;
      const int rr = (s == 0) ? 0 : p - 1;
      return (s == 0 ? -1.0 : 1.0) * sc.sx * sD[rr * p + k];
    }
    if (k != kb) return 0.0;
    const int rr = (s == 2) ? 0 : p - 1;
    return (s == 2 ? -1.0 : 1.0) * sc.sy * sD[rr * p + l];
  };
  if (Abi)
    for (int e = threadIdx.x; e < nb * ni; e += blockDim.x) {
      const int b = e / ni, c = e - b * ni;
      Abi[(size_t)leaf * nb * ni + e] = brow(b, c % m + 1, c / m + 1);
    }
  if (Abb)
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
      const int b = e / nb, b2 = e - b * nb;
      int k, l;
      bnode(b2, m, p, k, l);
      Abb[(size_t)leaf * nb * nb + e] = brow(b, k, l);
    }
}

__global__ void k_nodes(Geom g, const double *t, double *xy) {
  const int leaf = blockIdx.x, p = g.p;
  const double *b = g.box + 4 * (size_t)leaf;
  for (int n = threadIdx.x; n < p * p; n += blockDim.x) {
    const int i = n % p, j = n / p;
    xy[((size_t)leaf * p * p + n) * 2 + 0] = b[0] + (t[i] + 1.0) * (b[1] - b[0]) * 0.5;
    xy[((size_t)leaf * p * p + n) * 2 + 1] = b[2] + (t[j] + 1.0) * (b[3] - b[2]) * 0.5;
  }
}

__global__ void k_fill_int(int *dst, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}

__global__ void k_fill_double(double *dst, size_t n, double v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = v;
}

__global__ void k_copy_int(const int *src, int *dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

constexpr int kSolveNT = 256;

// Workgroup size of the factorisation: 4 waves when one wave factors the
// panel (R <= 256) so that several leaves share a CU; 8 waves otherwise.
inline int factor_nt(const Geom &g) { return g.R <= 256 ? 256 : 512; }

template <typename T>
size_t factor_lds(const Geom &g, int CH) {
  const int NW = factor_nt(g) / 64;
  size_t b = sizeof(T) * ((size_t)g.R * kPST + 16 * (size_t)(CH + 16) + 16 * kPST + 2 * NW);
  b += sizeof(int) * ((size_t)g.R + g.RT + 16 + 2 * NW + 1);
  return b;
}

constexpr size_t kLdsLimit = 160 * 1024;

// Column chunk of the U12 buffer: 128 columns for the small orders (keeps
// LDS low enough for several workgroups per CU), else as wide as fits.
template <typename T>
int pick_ch(const Geom &g) {
  const int full = g.CT * 16;
  if (g.tune_ch > 0) {
    const int c = g.tune_ch < full ? g.tune_ch : full;
    if (factor_lds<T>(g, c) <= kLdsLimit) return c;
  }
  const int top = g.R <= 256 ? 128 : 512;
  for (int ch = top; ch >= 16; ch -= 16) {
    const int c = ch < full ? ch : full;
    if (factor_lds<T>(g, c) <= kLdsLimit) return c;
  }
  return 0;
}


template <typename T>
size_t solve_lds(const Geom &g, int CW) {
  size_t b = sizeof(double) * (kSolveNT / 64);
  b += sizeof(T) * ((size_t)kSolveNB * 16 * (CW + 16) + 16 * kPST + 16 +
                    (size_t)kSolveNB * 16 * kPST);
  b += sizeof(int) * (2 * (size_t)g.R + g.RT);
  return b;
}

// Panels in pairs for R <= 256 (default); HPS_FACTOR_PAIRS=0 selects the
// one-panel-per-pass kernel.
bool factor_pairs_enabled() {
  static const bool on = [] {
    const char *v = std::getenv("HPS_FACTOR_PAIRS");
    return !(v && v[0] == '0');
  }();
  return on;
}

template <typename F>
hipError_t set_lds(F f, size_t bytes) {
  return hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace

size_t factor_lds_bytes(const Geom &g, bool fp32) {
  if (fp32) {
    const int ch = pick_ch<float>(g);
    return ch ? factor_lds<float>(g, ch) : 0;
  }
  const int ch = pick_ch<double>(g);
  return ch ? factor_lds<double>(g, ch) : 0;
}

template <typename T>
size_t factor2_lds(const Geom &g, int CH) {
  size_t b = sizeof(T) * (2 * (size_t)g.R * kPST + 32 * (size_t)(CH + 16) + 32 * kPST);
  b += sizeof(int) * ((size_t)g.R + g.RT + 33);
  return b;
}

// Column chunk of factor2: the largest multiple of 16 (at most 128) that
// leaves room for two workgroups per CU.
template <typename T>
int pick_ch2(const Geom &g) {
  const int full = g.CT * 16;
  if (g.tune_ch > 0) {
    const int c = g.tune_ch < full ? g.tune_ch : full;
    if (factor2_lds<T>(g, c) <= kLdsLimit) return c;
  }
  for (int ch = 128; ch >= 16; ch -= 16) {
    const int c = ch < full ? ch : full;
    if (factor2_lds<T>(g, c) <= kLdsLimit / 2) return c;
  }
  for (int ch = 128; ch >= 16; ch -= 16) {
    const int c = ch < full ? ch : full;
    if (factor2_lds<T>(g, c) <= kLdsLimit) return c;
  }
  return 0;
}

template <typename T>
hipError_t launch_factor2(const Geom &g, int nleaf, T *M, int *piv, int *rstep, int *info,
                          const BuildSrc &bs, hipStream_t s, const Sel &sel) {
  const int ch = pick_ch2<T>(g);
  if (!ch) return hipErrorInvalidValue;
  const size_t lds = factor2_lds<T>(g, ch);
  if constexpr (std::is_same<T, float>::value) {
    if (3 * lds <= kLdsLimit) {
    hipError_t e = set_lds(k_factor2_t<T, 3>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_factor2_t<T, 3>), dim3(nleaf), dim3(256), lds, s, g, M, piv, rstep, info,
                       ch, sel, bs);
    return hipGetLastError();
    }
  }
  hipError_t e = set_lds(k_factor2_t<T, 2>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_factor2_t<T, 2>), dim3(nleaf), dim3(256), lds, s, g, M, piv, rstep, info,
                     ch, sel, bs);
  return hipGetLastError();
}

template <typename T>
size_t factorP_lds(const Geom &g, int CH) {
  constexpr int NW = 512 / 64;
  size_t b = sizeof(T) * ((size_t)g.R * kPST + 32 * (size_t)(CH + 16) + 32 * kPST + 2 * NW);
  b += sizeof(int) * ((size_t)g.R + g.RT + 32 + 2 * NW + 1);
  return b;
}

// Column chunk of factorP: 128 columns if two workgroups then fit on a CU,
// else 64.  Each wavefront of the trailing pass takes strips of four column
// tiles, so chunks that are not a multiple of 64 leave a short strip per row
// tile that reloads the whole L21 operand (measured 10-20% slower).
template <typename T>
int pick_chP(const Geom &g) {
  const int full = g.CT * 16;
  if (g.tune_ch > 0) {
    const int c = g.tune_ch < full ? g.tune_ch : full;
    if (factorP_lds<T>(g, c) <= kLdsLimit) return c;
  }
  const int c128 = full < 128 ? full : 128, c64 = full < 64 ? full : 64;
  if (factorP_lds<T>(g, c128) <= kLdsLimit / 2) return c128;
  if (factorP_lds<T>(g, c64) <= kLdsLimit) return c64;
  for (int ch = 48; ch >= 16; ch -= 16) {
    const int c = ch < full ? ch : full;
    if (factorP_lds<T>(g, c) <= kLdsLimit) return c;
  }
  return 0;
}

// Two workgroups of 512 per CU need four wavefronts per SIMD (at most 128
// registers each) and half the LDS; the one-per-CU instance may use more
// registers.
template <typename T>
hipError_t launch_factorP(const Geom &g, int nleaf, T *M, int *piv, int *rstep, int *info,
                          const BuildSrc &bs, hipStream_t s, const Sel &sel) {
  const int ch = pick_chP<T>(g);
  if (!ch) return hipErrorInvalidValue;
  const size_t lds = factorP_lds<T>(g, ch);
  if (2 * lds <= kLdsLimit) {
    hipError_t e = set_lds(k_factorP<T, 512, 4>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_factorP<T, 512, 4>), dim3(nleaf), dim3(512), lds, s, g, M, piv, rstep,
                       info, ch, sel, bs);
    return hipGetLastError();
  }
  hipError_t e = set_lds(k_factorP<T, 512, 2>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_factorP<T, 512, 2>), dim3(nleaf), dim3(512), lds, s, g, M, piv, rstep, info,
                     ch, sel, bs);
  return hipGetLastError();
}

template <typename T>
size_t factor_ll_lds(const Geom &g, int NW, int RTW, int KT) {
  size_t b = sizeof(T) * (ll_panel_elems(g.R, NW, RTW) + 2 * 16 * 16 * (size_t)KT + 16 * kPST + 2 * NW);
  b += sizeof(int) * (4 * (size_t)g.R + 16 * (size_t)KT + 2 * NW + 1);
  return b;
}

template <typename T, int NW, int RTW, int MINB>
hipError_t launch_ll_t(const Geom &g, int nleaf, T *M, int *piv, int *rstep, int *info,
                       const BuildSrc &bs, hipStream_t s, const Sel &sel) {
  const size_t lds = factor_ll_lds<T>(g, NW, RTW, 2);
  if (lds > kLdsLimit || g.RT > NW * RTW) return hipErrorInvalidValue;
  hipError_t e = set_lds(k_factor_ll<T, NW, RTW, 2, MINB>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_factor_ll<T, NW, RTW, 2, MINB>), dim3(nleaf), dim3(64 * NW), lds, s, g,
                     M, piv, rstep, info, sel, bs);
  return hipGetLastError();
}

// Left-looking factorisation, 32-column block columns: up to 16 row tiles
// (R <= 256) with four wavefronts (one of them factors each panel in its
// registers) and two workgroups per CU; up to 64 row tiles with eight
// wavefronts.
template <typename T>
hipError_t launch_factor_ll(const Geom &g, int nleaf, T *M, int *piv, int *rstep, int *info,
                            const BuildSrc &bs, hipStream_t s, const Sel &sel) {
  if (g.RT <= 16) return launch_ll_t<T, 4, 4, 2>(g, nleaf, M, piv, rstep, info, bs, s, sel);
  return launch_ll_t<T, 8, 8, 1>(g, nleaf, M, piv, rstep, info, bs, s, sel);
}

template <int RT, int NW, int NS>
hipError_t launch_rr(const Geom &g, int nleaf, float *M, int *piv, int *rstep, int *info,
                     const BuildSrc &bs, hipStream_t s, const Sel &sel) {
  if (g.CT > NW * NS) return hipErrorNotSupported;
  hipLaunchKernelGGL((k_factor_rr<RT, NW, NS>), dim3(nleaf), dim3(64 * NW), 0, s, g, M, piv, rstep,
                     info, sel, bs);
  return hipGetLastError();
}

// Register-resident factorisation for the FP32 work matrices it covers
// (R <= 208); hipErrorNotSupported otherwise.  The (RT, wavefronts, column
// tiles per wavefront) instances cover p = 4 ... 16 with every right-hand
// side count the library uses.
hipError_t launch_factor_rr(const Geom &g, int nleaf, float *M, int *piv, int *rstep, int *info,
                            const BuildSrc &bs, hipStream_t s, const Sel &sel) {
  switch (g.RT) {
    case 1: return launch_rr<1, 4, 1>(g, nleaf, M, piv, rstep, info, bs, s, sel);
    case 2: return launch_rr<2, 4, 1>(g, nleaf, M, piv, rstep, info, bs, s, sel);
    case 3: return launch_rr<3, 4, 2>(g, nleaf, M, piv, rstep, info, bs, s, sel);
    case 4: return launch_rr<4, 4, 2>(g, nleaf, M, piv, rstep, info, bs, s, sel);
    case 6: return launch_rr<6, 8, 2>(g, nleaf, M, piv, rstep, info, bs, s, sel);
    case 7: return launch_rr<7, 8, 2>(g, nleaf, M, piv, rstep, info, bs, s, sel);
    case 8: return launch_rr<8, 8, 2>(g, nleaf, M, piv, rstep, info, bs, s, sel);
    case 9: return launch_rr<9, 8, 2>(g, nleaf, M, piv, rstep, info, bs, s, sel);
    case 11: return launch_rr<11, 8, 2>(g, nleaf, M, piv, rstep, info, bs, s, sel);
    case 13: return launch_rr<13, 4, 5>(g, nleaf, M, piv, rstep, info, bs, s, sel);
    default: return hipErrorNotSupported;
  }
}

// HPS_FACTOR_RR=0 turns the register-resident factorisation off.
bool factor_rr_enabled() {
  static const bool on = [] {
    const char *v = std::getenv("HPS_FACTOR_RR");
    return !(v && v[0] == '0');
  }();
  return on;
}

hipError_t launch_factor(const Geom &g, int nleaf, bool fp32, void *M, int *piv, int *rstep,
                         int *info, int mode, const double *f, const double *ub, hipStream_t s,
                         const Sel &sel) {
  const BuildSrc bs{mode, f, ub};
  // The left-looking factorisation is the default above 400 rows (p >= 23)
  // in both precisions, and in FP64 from 177 rows (p >= 16): measured 1.3x
  // (p = 24) to 1.5x (p = 32) faster than panel pairs for the whole
  // condensation, in FP32 1.3x at p = 32 (26.8 against 35.2 ms); in FP64
  // since the register-resident panels also 4.10 against 5.48 ms at p = 16
  // and 8.35 against 8.91 at p = 20, while FP32 stays slower there.
  if (g.tune_variant == 4 || (g.tune_variant == 0 && (g.R > 400 || (!fp32 && g.R > 176)))) {
    if (fp32) return launch_factor_ll<float>(g, nleaf, (float *)M, piv, rstep, info, bs, s, sel);
    return launch_factor_ll<double>(g, nleaf, (double *)M, piv, rstep, info, bs, s, sel);
  }
  if (fp32 && g.tune_variant == 3 && factor_rr_enabled()) {
    const hipError_t e = launch_factor_rr(g, nleaf, (float *)M, piv, rstep, info, bs, s, sel);
    if (e != hipErrorNotSupported) return e;
  }
  // An FP64 work matrix of 256 rows (p = 18) already pairs faster with one
  // panel in LDS (9.5 vs 12.0 ms for 4096 leaves), as do all larger ones.
  const bool large = g.R > 256 || (!fp32 && g.R == 256);
  const bool pairs = !large && g.tune_variant != 1 && factor_pairs_enabled();
  if (pairs) {
    if (fp32) return launch_factor2<float>(g, nleaf, (float *)M, piv, rstep, info, bs, s, sel);
    return launch_factor2<double>(g, nleaf, (double *)M, piv, rstep, info, bs, s, sel);
  }
  // FP32 work matrices below 400 rows run two single-panel workgroups per CU
  // without spills and gain nothing from pairs (measured at p = 19, 20)
  if (large && factor_pairs_enabled() &&
      (g.tune_variant == 2 || (g.tune_variant == 0 && (!fp32 || g.R >= 400)))) {
    if (fp32) return launch_factorP<float>(g, nleaf, (float *)M, piv, rstep, info, bs, s, sel);
    return launch_factorP<double>(g, nleaf, (double *)M, piv, rstep, info, bs, s, sel);
  }
  if (fp32) {
    const int ch = pick_ch<float>(g);
    if (!ch) return hipErrorInvalidValue;
    const size_t lds = factor_lds<float>(g, ch);
    if (factor_nt(g) == 256) {
      hipError_t e = set_lds(k_factor<float, 256>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_factor<float, 256>), dim3(nleaf), dim3(256), lds, s, g, (float *)M,
                         piv, rstep, info, ch, sel, bs);
    } else {
      hipError_t e = set_lds(k_factor<float, 512>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_factor<float, 512>), dim3(nleaf), dim3(512), lds, s, g, (float *)M,
                         piv, rstep, info, ch, sel, bs);
    }
  } else {
    const int ch = pick_ch<double>(g);
    if (!ch) return hipErrorInvalidValue;
    const size_t lds = factor_lds<double>(g, ch);
    if (factor_nt(g) == 256) {
      hipError_t e = set_lds(k_factor<double, 256>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_factor<double, 256>), dim3(nleaf), dim3(256), lds, s, g,
                         (double *)M, piv, rstep, info, ch, sel, bs);
    } else {
      hipError_t e = set_lds(k_factor<double, 512>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_factor<double, 512>), dim3(nleaf), dim3(512), lds, s, g,
                         (double *)M, piv, rstep, info, ch, sel, bs);
    }
  }
  return hipGetLastError();
}


template <int NT, int CW>
hipError_t launch_residual_t(const Geom &g, int nleaf, float *M32, const double *Xt,
                             const double *h, const double *f, const int *skip, double *norms,
                             int nch, hipStream_t s) {
  if (g.R > NT || nch < 1 || nch > kMaxChunks) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * (2 * (size_t)g.p * g.p + (size_t)CW * g.ni);
  hipError_t e = set_lds(k_residual<NT, CW>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_residual<NT, CW>), dim3(nleaf, nch), dim3(NT), lds, s, g, M32, Xt, h, f,
                     skip, norms);
  return hipGetLastError();
}

hipError_t launch_residual(const Geom &g, int nleaf, float *M32, const double *Xt,
                           const double *h, const double *f, const int *skip, double *norms,
                           int nch, hipStream_t s) {
  if (g.m <= 16 && g.R <= 256) {
    if (nch < 1 || nch > kMaxChunks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_residual_m, dim3(nleaf, nch), dim3(256), 0, s, g, M32, Xt, h, f, skip,
                       norms);
    return hipGetLastError();
  }
  // 2 x 2 tiles per grid: worth their padding from 24 nodes per line on
  // (measured 0.74x the thread-per-row kernel's speed at m = 18, 1.7x at
  // m = 30); a column must fit the 15 values per lane it stages
  if (g.m >= 24 && g.m <= 32 && g.ni <= 64 * 15) {
    if (nch < 1 || nch > kMaxChunks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_residual_m2, dim3(nleaf, nch), dim3(256), 0, s, g, M32, Xt, h, f, skip,
                       norms);
    return hipGetLastError();
  }
  if (g.R <= 256) return launch_residual_t<256, 8>(g, nleaf, M32, Xt, h, f, skip, norms, nch, s);
  return launch_residual_t<1024, 8>(g, nleaf, M32, Xt, h, f, skip, norms, nch, s);
}

template <typename T, int PASSES>
hipError_t launch_trisolve(const Geom &g, int nleaf, T *M, const int *piv, const int *rstep,
                           const BackOut &o, hipStream_t s, const Sel &sel, int nch = 1) {
  const int NRC = g.CT * 16 - g.R;
  const int cw = ((NRC / 16 + nch - 1) / nch) * 16;   // whole tiles per chunk
  const int nck = (NRC + cw - 1) / cw;
  if (nck != nch || nck > kMaxChunks) return hipErrorInvalidValue;
  const size_t lds = solve_lds<T>(g, cw);
  hipError_t e = set_lds(k_trisolve<T, kSolveNT, PASSES>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_trisolve<T, kSolveNT, PASSES>), dim3(nleaf, nck), dim3(kSolveNT), lds, s,
                     g, M, piv, rstep, o, sel, cw);
  return hipGetLastError();
}

// HPS_SOLVE_RR=0 turns the register-resident solves off.
bool solve_rr_enabled() {
  static const bool on = [] {
    const char *v = std::getenv("HPS_SOLVE_RR");
    return !(v && v[0] == '0');
  }();
  return on;
}

// The register-resident solves cover work matrices of at most 256 rows with
// at most five right-hand-side column tiles (every order p <= 18).
bool solve_rr_applies(const Geom &g) {
  const int nct = g.CT - g.RT;
  return solve_rr_enabled() && g.R <= 256 && nct >= 1 && nct <= 5;
}

template <typename T, int RTM, int NCTM, int NW, int MINW>
hipError_t launch_solve_rr_t(const Geom &g, int nleaf, const T *M, const int *piv,
                             const BackOut &o, hipStream_t s, const Sel &sel) {
  if (g.RT > RTM || g.CT - g.RT > NCTM) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * (8 + 2 * NCTM * 256) +
                     sizeof(T) * (size_t)g.RT * 16 * kDST + sizeof(int) * (size_t)g.R;
  hipError_t e = set_lds(k_solve_rr<T, RTM, NCTM, NW, MINW>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_solve_rr<T, RTM, NCTM, NW, MINW>), dim3(nleaf), dim3(64 * NW), lds,
                     s, g, M, piv, o, sel);
  return hipGetLastError();
}

// Up to 8 row tiles: four wavefronts, four per SIMD.  More: the FP64
// back substitution keeps four wavefronts (four row tiles each, up to 232
// registers, two wavefronts per SIMD), the FP32 one takes eight (at most
// 128 registers, four per SIMD); measured at p = 16 and 18.
template <typename T>
hipError_t launch_solve_rr(const Geom &g, int nleaf, const T *M, const int *piv, const BackOut &o,
                           hipStream_t s, const Sel &sel) {
  if (!solve_rr_applies(g)) return hipErrorNotSupported;
  constexpr bool wide = !std::is_same<T, double>::value;
  constexpr int NW = wide ? 8 : 4, MW = wide ? 4 : 2;
  const int nct = g.CT - g.RT;
  if (g.RT <= 4 && nct <= 4)
    return launch_solve_rr_t<T, 4, 4, 4, 4>(g, nleaf, M, piv, o, s, sel);
  if (g.RT <= 8 && nct <= 4)
    return launch_solve_rr_t<T, 8, 4, 4, 4>(g, nleaf, M, piv, o, s, sel);
  if (nct <= 4) return launch_solve_rr_t<T, 16, 4, NW, MW>(g, nleaf, M, piv, o, s, sel);
  return launch_solve_rr_t<T, 16, 5, NW, MW>(g, nleaf, M, piv, o, s, sel);
}

// HPS_BACKSOLVE_BIG=0 turns the register-resident solves of the work
// matrices above 256 rows off (the streaming solve then serves them).
// Measured (FP64 back substitution): 3.72 against 7.17 ms at 912 rows, 1.24
// against 1.78 ms at 336.
bool backsolve_big_enabled() {
  static const bool on = [] {
    const char *v = std::getenv("HPS_BACKSOLVE_BIG");
    return !(v && v[0] == '0');
  }();
  return on;
}

// The register-resident solves for work matrices above 256 rows: FP64
// factors (back substitution), and FP32 factors (back substitution, and the
// refinement correction's forward and backward passes in one launch).
bool solve_big_applies(const Geom &g) {
  return g.R > 256 && g.RT <= 8 * 8 && (size_t)g.R * 17 <= 8 * 8 * 256 &&
         (g.CT - g.RT + 1) / 2 <= kNormStride - 16 && backsolve_big_enabled();
}

template <typename T, int PASSES>
hipError_t launch_solve_big(const Geom &g, int nleaf, T *M, const int *piv, const BackOut &o,
                            hipStream_t s, const Sel &sel) {
  hipLaunchKernelGGL((k_inv_udiag<T, PASSES>), dim3(nleaf, (g.RT + 15) / 16), dim3(256), 0, s, g,
                     M, piv, sel);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = solve_big_lds<T, 8, 8>(g.R);
  if (lds > kLdsLimit) return hipErrorInvalidValue;
  e = set_lds(k_solve_big<T, 8, 8, PASSES>, lds);
  if (e != hipSuccess) return e;
  const int nck = (g.CT - g.RT + 1) / 2;
  const int groups = (nleaf + 7) / 8;
  hipLaunchKernelGGL((k_solve_big<T, 8, 8, PASSES>), dim3(groups * 8 * nck), dim3(512), lds, s,
                     g, (const T *)M, piv, o, sel, nleaf, nck);
  return hipGetLastError();
}

hipError_t launch_backsolve(const Geom &g, int nleaf, bool fp32, void *M, const int *piv,
                            const int *rstep, const BackOut &o, hipStream_t s, const Sel &sel) {
  if (solve_big_applies(g)) {
    if (fp32) return launch_solve_big<float, 1>(g, nleaf, (float *)M, piv, o, s, sel);
    return launch_solve_big<double, 1>(g, nleaf, (double *)M, piv, o, s, sel);
  }
  if (solve_rr_applies(g)) {
    if (fp32) return launch_solve_rr<float>(g, nleaf, (const float *)M, piv, o, s, sel);
    return launch_solve_rr<double>(g, nleaf, (const double *)M, piv, o, s, sel);
  }
  // two column chunks per leaf for the largest work matrices: twice the
  // reads of U, but twice the workgroups, each with half the LDS (FP64:
  // measured 7.17 against 8.55 ms at 912 rows; 2.10 against 1.78 ms at 336 rows)
  const int nch = (g.R > 512 && g.CT - g.RT >= 2) ? 2 : 1;
  if (fp32) return launch_trisolve<float, 1>(g, nleaf, (float *)M, piv, rstep, o, s, sel, nch);
  return launch_trisolve<double, 1>(g, nleaf, (double *)M, piv, rstep, o, s, sel, nch);
}

template <int RTM>
hipError_t launch_solve_cols_t(const Geom &g, int nleaf, const float *M, const int *piv,
                               const BackOut &o, hipStream_t s) {
  if (g.RT > RTM) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * 8 + sizeof(float) * (size_t)g.RT * 16 * kDST +
                     sizeof(int) * (size_t)g.R;
  hipError_t e = set_lds(k_solve_cols<RTM>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_solve_cols<RTM>), dim3(nleaf), dim3(64 * (g.CT - g.RT)), lds, s, g, M,
                     piv, o);
  return hipGetLastError();
}

hipError_t launch_solve_cols(const Geom &g, int nleaf, const float *M, const int *piv,
                             const BackOut &o, hipStream_t s) {
  if (g.RT <= 4) return launch_solve_cols_t<4>(g, nleaf, M, piv, o, s);
  if (g.RT <= 8) return launch_solve_cols_t<8>(g, nleaf, M, piv, o, s);
  if (g.RT <= 13) return launch_solve_cols_t<13>(g, nleaf, M, piv, o, s);
  return launch_solve_cols_t<16>(g, nleaf, M, piv, o, s);
}

hipError_t launch_refine_solve(const Geom &g, int nleaf, void *M, const int *piv,
                               const int *rstep, const BackOut &o, int nch, hipStream_t s) {
  if (solve_rr_applies(g)) {
    if (nch != 1) return hipErrorInvalidValue;
    return launch_solve_cols(g, nleaf, (const float *)M, piv, o, s);
  }
  if (solve_big_applies(g)) return launch_solve_big<float, 3>(g, nleaf, (float *)M, piv, o, s, Sel());
  return launch_trisolve<float, 3>(g, nleaf, (float *)M, piv, rstep, o, s, Sel(), nch);
}

int refine_solve_chunks(const Geom &g, int nch) {
  if (solve_rr_applies(g)) return 1;
  if (solve_big_applies(g)) return (g.CT - g.RT + 1) / 2;
  return nch;
}

// The first two refinement iterations cover every leaf, or about half of
// them on the hardest workloads, in one workgroup each (splitting would only
// re-read the factors); later ones are left with the few leaves still
// refining, so their columns are split over up to four workgroups (the
// chunk count is the number of 16-column tiles the solve splits into, at
// most four).  The register-resident solves already spread a leaf's column
// tiles over the wavefronts of its one workgroup.
int refine_chunks(const Geom &g, int it) {
  if (solve_rr_applies(g)) return 1;
  if (it <= 1) return (g.R > 512 && g.CT - g.RT >= 2) ? 2 : 1;   // as the back substitution
  const int tiles = (g.CT * 16 - g.R) / 16;
  const int per = (tiles + kMaxChunks - 1) / kMaxChunks;   // tiles per chunk
  return (tiles + per - 1) / per;
}

hipError_t launch_convcheck(int nleaf, double *norms, double tol, int *conv, int *info, int it,
                            int last, int nres, int nsol, hipStream_t s) {
  hipLaunchKernelGGL(k_convcheck, dim3((nleaf + 255) / 256), dim3(256), 0, s, nleaf, norms, tol,
                     conv, info, it, last, nres, nsol);
  return hipGetLastError();
}

hipError_t launch_collect(int nleaf, int *info, int *list, int *count, int *total, int *redo,
                          hipStream_t s) {
  if (nleaf <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_collect, dim3((nleaf + 255) / 256), dim3(256), 0, s, nleaf, info, list,
                     count, total, redo);
  return hipGetLastError();
}

hipError_t launch_schur(const Geom &g, int nleaf, const double *Xt, const double *h, double *S,
                        double *w, int *info, hipStream_t s) {
  // sixteen columns per pass while that keeps LDS under 32 KB, else eight
  const int cols = g.ni * 16 * sizeof(double) <= 32 * 1024 ? 16 : 8;
  const size_t lds = sizeof(double) * cols * (size_t)g.ni;
  hipError_t e = set_lds(k_schur, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_schur, dim3(nleaf), dim3(256), lds, s, g, Xt, h, S, w, info, cols);
  return hipGetLastError();
}

hipError_t launch_recover(const Geom &g, int nleaf, const double *Xt, const double *h,
                          const double *ub, double *ui, hipStream_t s) {
  hipLaunchKernelGGL(k_recover, dim3(nleaf, (g.ni + 255) / 256), dim3(256), 0, s, g, Xt, h, ub, ui);
  return hipGetLastError();
}

hipError_t launch_operator(const Geom &g, int nleaf, double *Aii, double *Aib, double *Abi,
                           double *Abb, hipStream_t s) {
  hipLaunchKernelGGL(k_operator, dim3(nleaf), dim3(256), 0, s, g, Aii, Aib, Abi, Abb);
  return hipGetLastError();
}

hipError_t launch_nodes(const Geom &g, int nleaf, const double *t, double *xy, hipStream_t s) {
  hipLaunchKernelGGL(k_nodes, dim3(nleaf), dim3(256), 0, s, g, t, xy);
  return hipGetLastError();
}

hipError_t launch_fill_int(int *dst, int n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, dst, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_double(double *dst, size_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_double, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, n, v);
  return hipGetLastError();
}

hipError_t launch_copy_info(const int *src, int *dst, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_int, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace hps
