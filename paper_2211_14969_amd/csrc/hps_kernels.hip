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
// Elimination (Sec. 2: "LU factorization, matrix-matrix multiply" on every
// leaf) is a right-looking blocked LU with partial pivoting over panels of
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
#include <climits>
#include <cmath>
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
template <>
struct Mfma<float> {
  using acc = f4;
  __device__ static __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Element (r, c) of a tile-major work matrix with CT column tiles.  Inside a
// 16 x 16 tile the 256 elements are ordered as the accumulator registers of
// the 16x16x4 MFMA instruction of that precision: element q*64 + lane holds
// accumulator register q of that lane.  The two precisions differ (checked
// on gfx950 with a one-hot probe of the builtins):
//   f32: row r in register r%4 of lanes 16*(r/4) .. +15, column = lane%16;
//   f64: row r in register r/4 of lanes 16*(r%4) .. +15, column = lane%16,
//        which is plain row-major order within the tile.
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
struct Tile<float> {
  __device__ static __forceinline__ int inner(int r, int c) {
    return ((r & 3) << 6) + (((r >> 2) & 3) << 4) + (c & 15);
  }
  __device__ static __forceinline__ int crow(int q, int lane) { return 4 * (lane >> 4) + q; }
  __device__ static __forceinline__ void rc(int w, int &r, int &c) {
    const int q = w >> 6, ln = w & 63;
    r = 4 * (ln >> 4) + q;
    c = ln & 15;
  }
};

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

__device__ __forceinline__ size_t leaf_stride(const Geom &g) {
  return (size_t)g.RT * g.CT * 256;
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
// diagonal, with d1 = (2/hx) D, d11 = (2/hx)^2 D^2 (likewise in x2).
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
  return v;
}

__device__ __forceinline__ void stage_tables(const Geom &g, double *sD, double *sD2) {
  const int pp = g.p * g.p;
  for (int e = threadIdx.x; e < pp; e += blockDim.x) {
    sD[e] = g.D[e];
    sD2[e] = g.D2[e];
  }
}

// ---------------------------------------------------------------------------
// build: form W = [A_ii | rhs] of every leaf (operator step of Sec. 2)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_build(Geom g, int mode, T *M, const double *f,
                                               const double *ub, Sel sel) {
  __shared__ double sD[32 * 32], sD2[32 * 32];
  int leaf;
  if (!resolve_leaf(sel, leaf)) return;
  stage_tables(g, sD, sD2);
  __syncthreads();
  const LeafScale sc = leaf_scale(g, leaf);
  const int p = g.p, m = g.m, ni = g.ni, nb = g.nb, R = g.R, CT = g.CT;
  const size_t nbase = (size_t)leaf * p * p;
  T *Ml = M + leaf_stride(g) * blockIdx.x;
  const size_t total = leaf_stride(g);
  for (size_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int tile = (int)(e >> 8);
    int ri, ci;
    Tile<T>::rc((int)(e & 255), ri, ci);
    const int r = (tile / CT) * 16 + ri;
    const int c = (tile % CT) * 16 + ci;
    double v = 0.0;
    if (r >= ni) {
      v = (c == r) ? 1.0 : 0.0;
    } else {
      const int i = r % m + 1, j = r / m + 1;
      if (c < ni) {
        v = opval(g, sD, sD2, sc, nbase, i, j, c % m + 1, c / m + 1);
      } else if (c >= R) {
        const int jr = c - R;
        if (mode == RHS_CONDENSE) {
          if (jr < nb) {
            int k, l;
            bnode(jr, m, p, k, l);
            v = opval(g, sD, sD2, sc, nbase, i, j, k, l);
          } else if (jr == nb && f) {
            v = f[(size_t)leaf * ni + r];
          }
        } else if (jr == 0) {  // RHS_REFACTOR: f_i - A_ib u_b
          const double *u = ub + (size_t)leaf * nb;
          v = f ? f[(size_t)leaf * ni + r] : 0.0;
          v -= opval(g, sD, sD2, sc, nbase, i, j, 0, j) * u[j - 1];
          v -= opval(g, sD, sD2, sc, nbase, i, j, p - 1, j) * u[m + j - 1];
          v -= opval(g, sD, sD2, sc, nbase, i, j, i, 0) * u[2 * m + i - 1];
          v -= opval(g, sD, sD2, sc, nbase, i, j, i, p - 1) * u[3 * m + i - 1];
        }
      }
    }
    Ml[e] = (T)v;
  }
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

template <typename T, int NT>
__global__ void __launch_bounds__(NT, 512 / NT) k_factor(Geom g, T *M, int *piv, int *rstep,
                                               int *info, int CH, Sel sel) {
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
  T *redv = Linv + 16 * kPST;             // [NW]
  int *rst = (int *)(redv + NW);          // [R]         retire step
  int *tileAct = rst + R;                 // [RT]
  int *pv = tileAct + RT;                 // [16]
  int *redi = pv + 16;                    // [NW]
  int *zeroPiv = redi + NW;               // [1]
  T *Ml = M + leaf_stride(g) * wi;

  for (int r = tid; r < R; r += NT) rst[r] = kInfoActive;
  if (tid == 0) *zeroPiv = 0;
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
      for (int c = 0; c < 16; ++c) {
        T best = T(-1);
        int bi = INT_MAX;
        for (int r = tid; r < R; r += NT) {
          if (rst[r] != kInfoActive) continue;
          const T v = abs_key(P[r * kPST + c]);
          if (v > best) { best = v; bi = r; }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const T ob = __shfl_xor(best, off);
          const int oi = __shfl_xor(bi, off);
          if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (lane == 0) { redv[wv] = best; redi[wv] = bi; }
        __syncthreads();
        best = redv[0];
        bi = redi[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) {
          const T ob = redv[w];
          const int oi = redi[w];
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
        for (int r = tid; r < R; r += NT) {
          if (r == pr || rst[r] != kInfoActive) continue;
          const T l = P[r * kPST + c] * inv;
          P[r * kPST + c] = l;
          for (int cc = c + 1; cc < 16; ++cc) P[r * kPST + cc] -= l * P[pr * kPST + cc];
        }
        __syncthreads();
      }
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

// Right-hand-side update of the triangular solves:  C -= A * Y for every
// row tile with a qualifying row, where A = W[rows, panel k] (rows retired
// after step k for the forward replay, before it for the back substitution;
// other rows contribute zero) and Y the 16 solved rows in LDS.  Each wave
// takes a row tile and up to four right-hand-side tiles at once.
template <typename T, int NW>
__device__ __forceinline__ void strip_update(T *Ml, const T *Y, int YST, const int *rst,
                                             const int *tileAny, int RT, int CT, int R, int ntj,
                                             int k, bool after, int wv, int lane) {
  const int nstrip = (ntj + 3) >> 2;
  for (int t = wv; t < RT * nstrip; t += NW) {
    const int ti = t / nstrip, j0 = (t - ti * nstrip) * 4;
    if (!tileAny[ti]) continue;
    const int nj = min(4, ntj - j0);
    T *Ct = Ml + ((size_t)(ti * CT + (R >> 4) + j0) << 8);
    typename Mfma<T>::acc acc[4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      if (jj < nj) {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[jj][q] = Ct[jj * 256 + q * 64 + lane];
      }
    }
    const int ar = ti * 16 + (lane & 15);
    const bool use = after ? rst[ar] > k : rst[ar] < k;
    T a[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
      a[kc] = use ? -Ml[tix<T>(ar, k * 16 + 4 * kc + (lane >> 4), CT)] : T(0);
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      if (jj < nj) {
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
          const T b = Y[(4 * kc + (lane >> 4)) * YST + (j0 + jj) * 16 + (lane & 15)];
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
}

// ---------------------------------------------------------------------------
// forward replay of the stored L on fresh right-hand sides (refinement)
// ---------------------------------------------------------------------------
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_fwdsolve(Geom g, T *M, const int *piv,
                                                 const int *rstep, const int *skip) {
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  const int leaf = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (skip && skip[leaf]) return;
  const int R = g.R, RT = g.RT, CT = g.CT, NRC = CT * 16 - R, YST = NRC + 16;
  T *Y = (T *)smem;                 // [16][YST]
  T *Lt = Y + 16 * YST;             // [16][kPST]
  int *rst = (int *)(Lt + 16 * kPST);
  int *tileAny = rst + R;
  int *pv = tileAny + RT;
  T *Ml = M + leaf_stride(g) * leaf;
  for (int r = tid; r < R; r += NT) rst[r] = rstep[(size_t)leaf * R + r];
  for (int k = 0; k < RT; ++k) {
    if (tid < 16) pv[tid] = piv[(size_t)leaf * R + k * 16 + tid];
    __syncthreads();
    for (int e = tid; e < 256; e += NT) {
      const int s = e >> 4, q = e & 15;
      Lt[s * kPST + q] = Ml[tix<T>(pv[s], k * 16 + q, CT)];
    }
    for (int t = tid; t < RT; t += NT) {
      int a = 0;
      for (int q = 0; q < 16; ++q) a |= (rst[t * 16 + q] > k);
      tileAny[t] = a;
    }
    __syncthreads();
    for (int jr = tid; jr < NRC; jr += NT) {
      T u[16];
#pragma unroll
      for (int s = 0; s < 16; ++s) u[s] = Ml[tix<T>(pv[s], R + jr, CT)];
#pragma unroll
      for (int s = 1; s < 16; ++s) {
        T acc = u[s];
#pragma unroll
        for (int q = 0; q < s; ++q) acc -= Lt[s * kPST + q] * u[q];
        u[s] = acc;
      }
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        Y[s * YST + jr] = u[s];
        Ml[tix<T>(pv[s], R + jr, CT)] = u[s];
      }
    }
    __syncthreads();
    strip_update<T, NW>(Ml, Y, YST, rst, tileAny, RT, CT, R, NRC >> 4, k, /*after=*/true, wv,
                        lane);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// back substitution U X = Y over the right-hand-side columns
// ---------------------------------------------------------------------------
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_backsolve(Geom g, T *M, const int *piv,
                                                  const int *rstep, BackOut o, Sel sel) {
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  const int wi = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int leaf;
  if (!resolve_leaf(sel, leaf)) return;
  if (o.skip && o.skip[leaf]) return;
  const int R = g.R, RT = g.RT, CT = g.CT, ni = g.ni, nb = g.nb;
  const int NRC = CT * 16 - R, YST = NRC + 16;
  double *red = (double *)smem;     // [NW]
  T *Y = (T *)(red + NW);           // [16][YST]
  T *Ut = Y + 16 * YST;             // [16][kPST]
  int *rst = (int *)(Ut + 16 * kPST);
  int *tileAny = rst + R;
  int *pv = tileAny + RT;
  T *Ml = M + leaf_stride(g) * wi;
  double nd = 0.0;
  for (int r = tid; r < R; r += NT) rst[r] = rstep[(size_t)wi * R + r];
  for (int k = RT - 1; k >= 0; --k) {
    if (tid < 16) pv[tid] = piv[(size_t)wi * R + k * 16 + tid];
    __syncthreads();
    for (int e = tid; e < 256; e += NT) {
      const int s = e >> 4, q = e & 15;
      Ut[s * kPST + q] = Ml[tix<T>(pv[s], k * 16 + q, CT)];
    }
    for (int e = tid; e < 16 * NRC; e += NT) {
      const int s = e / NRC, jr = e - s * NRC;
      Y[s * YST + jr] = Ml[tix<T>(pv[s], R + jr, CT)];
    }
    for (int t = tid; t < RT; t += NT) {
      int a = 0;
      for (int q = 0; q < 16; ++q) a |= (rst[t * 16 + q] < k);
      tileAny[t] = a;
    }
    __syncthreads();
    for (int jr = tid; jr < NRC; jr += NT) {
      T x[16];
#pragma unroll
      for (int s = 15; s >= 0; --s) {
        T acc = Y[s * YST + jr];
#pragma unroll
        for (int q = s + 1; q < 16; ++q) acc -= Ut[s * kPST + q] * x[q];
        x[s] = acc / Ut[s * kPST + s];
      }
#pragma unroll
      for (int s = 0; s < 16; ++s) Y[s * YST + jr] = x[s];
      if (jr < g.nrhs) {
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          const int i = k * 16 + s;
          if (i >= ni) continue;
          const double v = (double)x[s];
          if (o.mode == BACK_UI) {
            o.ui[(size_t)leaf * ni + i] = v;
          } else {
            double *dst = (jr < nb) ? o.Xt + ((size_t)leaf * nb + jr) * ni + i
                                    : o.h + (size_t)leaf * ni + i;
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
    if (k > 0) {
      strip_update<T, NW>(Ml, Y, YST, rst, tileAny, RT, CT, R, NRC >> 4, k, /*after=*/false, wv,
                          lane);
      __syncthreads();
    }
  }
  if (o.mode == BACK_ACCUM) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) nd += __shfl_xor(nd, off);
    if (lane == 0) red[wv] = nd;
    __syncthreads();
    if (tid == 0) {
      double a = 0.0;
      for (int w = 0; w < NW; ++w) a += red[w];
      o.norms[8 * (size_t)leaf + 5] = a;
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 refinement residual  r = A_ib - A_ii X  (and f_i - A_ii h), applied
// through the tensor structure of the collocation operator: each interior
// row couples only to its own x1-line and x2-line of nodes.  The residual is
// written in FP32 into the right-hand-side columns of the work matrix for the
// correction solve, and the squared Frobenius norms of r, X, A_ii and
// [A_ib f_i] are stored per leaf for the backward-error stop test.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_residual(Geom g, float *M32, const double *Xt,
                                                  const double *h, const double *f,
                                                  const int *skip, double *norms) {
  __shared__ double sD[32 * 32], sD2[32 * 32];
  __shared__ double xcol[30 * 30];
  __shared__ double red[4][4];
  const int leaf = blockIdx.x;
  if (skip && skip[leaf]) return;
  stage_tables(g, sD, sD2);
  const LeafScale sc = leaf_scale(g, leaf);
  const int p = g.p, m = g.m, ni = g.ni, nb = g.nb, R = g.R, CT = g.CT;
  const size_t nbase = (size_t)leaf * p * p;
  float *Ml = M32 + leaf_stride(g) * leaf;
  const int ncol = (h && f) ? nb + 1 : nb;
  double nr = 0.0, nx = 0.0, na = 0.0, nbb = 0.0;
  for (int jr = 0; jr < ncol; ++jr) {
    __syncthreads();
    const double *src = (jr < nb) ? Xt + ((size_t)leaf * nb + jr) * ni : h + (size_t)leaf * ni;
    for (int e = threadIdx.x; e < ni; e += blockDim.x) xcol[e] = src[e];
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
      double res = 0.0;
      if (r < ni) {
        const int i = r % m + 1, j = r / m + 1;
        const size_t n = nbase + i + (size_t)p * j;
        const double a11 = g.a11 ? g.a11[n] : 1.0, c1 = g.c1 ? g.c1[n] : 0.0;
        const double a22 = g.a22 ? g.a22[n] : 1.0, c2 = g.c2 ? g.c2[n] : 0.0;
        const double k2b = g.k2b ? g.k2b[n] : 0.0;
        const double ax2 = a11 * sc.sx * sc.sx, ax1 = c1 * sc.sx;
        const double ay2 = a22 * sc.sy * sc.sy, ay1 = c2 * sc.sy;
        double ax = -k2b * xcol[r];
        for (int k = 1; k <= m; ++k)
          ax -= (ax2 * sD2[i * p + k] + ax1 * sD[i * p + k]) * xcol[(k - 1) + m * (j - 1)];
        for (int l = 1; l <= m; ++l)
          ax -= (ay2 * sD2[j * p + l] + ay1 * sD[j * p + l]) * xcol[(i - 1) + m * (l - 1)];
        double bval;
        if (jr < nb) {
          int k, l;
          bnode(jr, m, p, k, l);
          bval = opval(g, sD, sD2, sc, nbase, i, j, k, l);
        } else {
          bval = f[(size_t)leaf * ni + r];
        }
        res = bval - ax;
        nr += res * res;
        nx += xcol[r] * xcol[r];
        nbb += bval * bval;
        if (jr == 0) {
          // squared norm of row r of A_ii: off-diagonal x1- and x2-line
          // entries, and the diagonal where both lines and k2b meet
          double diag = -k2b;
          for (int k = 1; k <= m; ++k) {
            const double v = -(ax2 * sD2[i * p + k] + ax1 * sD[i * p + k]);
            if (k == i) diag += v; else na += v * v;
          }
          for (int l = 1; l <= m; ++l) {
            const double v = -(ay2 * sD2[j * p + l] + ay1 * sD[j * p + l]);
            if (l == j) diag += v; else na += v * v;
          }
          na += diag * diag;
        }
      }
      Ml[tix<float>(r, R + jr, CT)] = (float)res;
    }
  }
  // block reduction of the four sums
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    nr += __shfl_xor(nr, off);
    nx += __shfl_xor(nx, off);
    na += __shfl_xor(na, off);
    nbb += __shfl_xor(nbb, off);
  }
  if (lane == 0) {
    red[wv][0] = nr;
    red[wv][1] = nx;
    red[wv][2] = na;
    red[wv][3] = nbb;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double a = 0.0;
    for (int w = 0; w < 4; ++w) a += red[w][threadIdx.x];
    norms[8 * (size_t)leaf + threadIdx.x] = a;
  }
}

// Stop test of the refinement, per leaf, after the residual r_k of X_k:
//  * the normwise backward error ||r||/(||A_ii|| ||X|| + ||[A_ib f]||) is at
//    the FP64 rounding level, or
//  * the estimated forward error (||r_k|| / ||r_{k-1}||) ||dX_k||, i.e. the
//    observed contraction of the residual times the last correction, is at
//    most tol ||X_k||.
// On the final check a leaf that passed neither is flagged -1.
// norms[8l + ...]: 0 ||r||^2, 1 ||X||^2, 2 ||A_ii||^2, 3 ||[A_ib f]||^2,
// 4 previous ||r||^2, 5 ||dX||^2 of the last correction.
__global__ void k_convcheck(int nleaf, double *norms, double tol, int *conv, int *info,
                            int it, int last) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nleaf || conv[l]) return;
  double *n = norms + 8 * (size_t)l;
  const double eta = sqrt(n[0]) / (sqrt(n[2]) * sqrt(n[1]) + sqrt(n[3]));
  bool ok = eta <= 4.0 * 0x1p-53;
  if (!ok && it > 0 && n[4] > 0.0) {
    const double est = sqrt(n[0] / n[4]) * sqrt(n[5]);
    ok = est <= tol * sqrt(n[1]);
  }
  n[4] = n[0];
  if (ok) {
    conv[l] = 1;
  } else if (last && info[l] == 0) {
    info[l] = -1;
  }
}

// Leaves whose refinement failed (info -1) are listed for an FP64 redo.
__global__ void k_collect(int nleaf, int *info, int *list, int *count, int *total) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nleaf || info[l] != -1) return;
  atomicAdd(total, 1);
  const int slot = atomicAdd(count, 1);
  list[slot] = l;
  info[l] = 0;
}

// ---------------------------------------------------------------------------
// Schur complement S = A_bb - A_bi X and w = A_bi h in FP64.  A_bi has p-2
// nonzeros per row (the normal derivative along one grid line) and A_bb two.
// Columns of X are staged through LDS a few at a time so that every global
// read is coalesced.
// ---------------------------------------------------------------------------
constexpr int kSchurCols = 8;

__global__ void __launch_bounds__(256) k_schur(Geom g, const double *Xt, const double *h,
                                               double *S, double *w, int *info) {
  __shared__ double sD0[32], sD1[32];   // rows 0 and p-1 of D
  __shared__ double xs[kSchurCols * 900];
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
    for (int e = threadIdx.x; e < cw * ni; e += blockDim.x) {
      const int c = e / ni, i = e - c * ni;
      const int col = c0 + c;
      double v = 0.0;
      if (col < nb) v = Xl[(size_t)col * ni + i];
      else if (h) v = h[(size_t)leaf * ni + i];
      xs[c * ni + i] = v;
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
      int k, l;
      bnode(b, m, p, k, l);
      Aib[(size_t)leaf * ni * nb + e] = opval(g, sD, sD2, sc, nbase, r % m + 1, r / m + 1, k, l);
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
  size_t b = sizeof(T) * ((size_t)g.R * kPST + 16 * (size_t)(CH + 16) + 16 * kPST + NW);
  b += sizeof(int) * ((size_t)g.R + g.RT + 16 + NW + 1);
  return b;
}

constexpr size_t kLdsLimit = 160 * 1024;

// Column chunk of the U12 buffer: 128 columns for the small orders (keeps
// LDS low enough for several workgroups per CU), else as wide as fits.
template <typename T>
int pick_ch(const Geom &g) {
  const int full = g.CT * 16;
  const int top = g.R <= 256 ? 128 : 512;
  for (int ch = top; ch >= 16; ch -= 16) {
    const int c = ch < full ? ch : full;
    if (factor_lds<T>(g, c) <= kLdsLimit) return c;
  }
  return 0;
}

template <typename T>
size_t solve_lds(const Geom &g) {
  const int NRC = g.CT * 16 - g.R;
  size_t b = sizeof(double) * (kSolveNT / 64);
  b += sizeof(T) * (16 * (size_t)(NRC + 16) + 16 * kPST);
  b += sizeof(int) * ((size_t)g.R + g.RT + 16);
  return b;
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

hipError_t launch_build(const Geom &g, int nleaf, int mode, bool fp32, void *M,
                        const double *f, const double *ub, hipStream_t s, const Sel &sel) {
  if (fp32)
    hipLaunchKernelGGL(k_build<float>, dim3(nleaf), dim3(256), 0, s, g, mode, (float *)M, f, ub,
                       sel);
  else
    hipLaunchKernelGGL(k_build<double>, dim3(nleaf), dim3(256), 0, s, g, mode, (double *)M, f, ub,
                       sel);
  return hipGetLastError();
}

hipError_t launch_factor(const Geom &g, int nleaf, bool fp32, void *M, int *piv, int *rstep,
                         int *info, hipStream_t s, const Sel &sel) {
  if (fp32) {
    const int ch = pick_ch<float>(g);
    if (!ch) return hipErrorInvalidValue;
    const size_t lds = factor_lds<float>(g, ch);
    if (factor_nt(g) == 256) {
      hipError_t e = set_lds(k_factor<float, 256>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_factor<float, 256>), dim3(nleaf), dim3(256), lds, s, g, (float *)M,
                         piv, rstep, info, ch, sel);
    } else {
      hipError_t e = set_lds(k_factor<float, 512>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_factor<float, 512>), dim3(nleaf), dim3(512), lds, s, g, (float *)M,
                         piv, rstep, info, ch, sel);
    }
  } else {
    const int ch = pick_ch<double>(g);
    if (!ch) return hipErrorInvalidValue;
    const size_t lds = factor_lds<double>(g, ch);
    if (factor_nt(g) == 256) {
      hipError_t e = set_lds(k_factor<double, 256>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_factor<double, 256>), dim3(nleaf), dim3(256), lds, s, g,
                         (double *)M, piv, rstep, info, ch, sel);
    } else {
      hipError_t e = set_lds(k_factor<double, 512>, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_factor<double, 512>), dim3(nleaf), dim3(512), lds, s, g,
                         (double *)M, piv, rstep, info, ch, sel);
    }
  }
  return hipGetLastError();
}

hipError_t launch_backsolve(const Geom &g, int nleaf, bool fp32, void *M, const int *piv,
                            const int *rstep, const BackOut &o, hipStream_t s, const Sel &sel) {
  if (fp32) {
    const size_t lds = solve_lds<float>(g);
    hipError_t e = set_lds(k_backsolve<float, kSolveNT>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_backsolve<float, kSolveNT>), dim3(nleaf), dim3(kSolveNT), lds, s, g,
                       (float *)M, piv, rstep, o, sel);
  } else {
    const size_t lds = solve_lds<double>(g);
    hipError_t e = set_lds(k_backsolve<double, kSolveNT>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_backsolve<double, kSolveNT>), dim3(nleaf), dim3(kSolveNT), lds, s, g,
                       (double *)M, piv, rstep, o, sel);
  }
  return hipGetLastError();
}

hipError_t launch_fwdsolve(const Geom &g, int nleaf, bool fp32, void *M, const int *piv,
                           const int *rstep, const int *skip, hipStream_t s) {
  if (fp32) {
    const size_t lds = solve_lds<float>(g);
    hipError_t e = set_lds(k_fwdsolve<float, kSolveNT>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fwdsolve<float, kSolveNT>), dim3(nleaf), dim3(kSolveNT), lds, s, g,
                       (float *)M, piv, rstep, skip);
  } else {
    const size_t lds = solve_lds<double>(g);
    hipError_t e = set_lds(k_fwdsolve<double, kSolveNT>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fwdsolve<double, kSolveNT>), dim3(nleaf), dim3(kSolveNT), lds, s, g,
                       (double *)M, piv, rstep, skip);
  }
  return hipGetLastError();
}

hipError_t launch_residual(const Geom &g, int nleaf, float *M32, const double *Xt,
                           const double *h, const double *f, const int *skip, double *norms,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(nleaf), dim3(256), 0, s, g, M32, Xt, h, f, skip, norms);
  return hipGetLastError();
}

hipError_t launch_convcheck(int nleaf, double *norms, double tol, int *conv, int *info, int it,
                            int last, hipStream_t s) {
  hipLaunchKernelGGL(k_convcheck, dim3((nleaf + 255) / 256), dim3(256), 0, s, nleaf, norms, tol,
                     conv, info, it, last);
  return hipGetLastError();
}

hipError_t launch_collect(int nleaf, int *info, int *list, int *count, int *total,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_collect, dim3((nleaf + 255) / 256), dim3(256), 0, s, nleaf, info, list,
                     count, total);
  return hipGetLastError();
}

hipError_t launch_schur(const Geom &g, int nleaf, const double *Xt, const double *h, double *S,
                        double *w, int *info, hipStream_t s) {
  hipLaunchKernelGGL(k_schur, dim3(nleaf), dim3(256), 0, s, g, Xt, h, S, w, info);
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
