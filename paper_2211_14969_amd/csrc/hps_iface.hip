// FP64 direct solve of the reduced interface system (eq. (hps_reduced)) in
// nested-dissection order, the first of the two solvers of Sec. 2.
//
// Planning (host): the nx x ny leaf grid is bisected recursively, the longer
// side first.  A box's exterior list E holds the unknown edge nodes on its
// boundary (nodes on the outer boundary carry Dirichlet data and are never
// unknowns).  Bisecting box b into halves a and c, the separator s is the
// set of nodes both halves have on their boundary (the leaf edges along the
// cut), and E_b = (E_a \ s) ++ (E_c \ s).  A leaf's exterior lists its unknown
// boundary slots, and its Schur complement is its own S restricted to them.
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
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/hps_iface.h"
#include "hps_internal.h"

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kMaxSep = HPS_IFACE_MAX_SEPARATOR;
constexpr int kFactorThreads = 512;   // LU of one separator block per workgroup
constexpr int kSolveThreads = 512;    // 16 right-hand sides per workgroup

// One front as the kernels see it.  Arena offsets are in doubles (FP64
// arena) or ints (int arena).  A child that is a leaf is coded as -(leaf+1):
// its Schur complement is S + leaf*nb*nb (leading dimension nb) and its
// reduced right-hand side the leaf's row of the leaf right-hand sides.
struct Front {
  long long fss, x, fes, t, y, r;
  long long ca, cc;   // children's Schur complements
  long long ra, rc;   // children's reduced right-hand sides
  int lda, ldc;       // leading dimensions of the children's Schur complements
  int map;            // int arena: map_a [nS+nE], then map_c [nS+nE]
  int gid;            // int arena: global node ids, separator then exterior
  int perm;           // int arena: pivot order of the LU of F_ss [nS]
  int nS, nE;
};

// Global id of slot s of leaf t, and whether it lies on the outer boundary.
// Edge ids: vertical edges (line ix = 0..nx, row iy) first, then horizontal
// ones (column ix, line iy = 0..ny); node k of an edge is id * m + k.
__host__ __device__ inline int leaf_node(int nx, int ny, int m, int t, int s, bool &dir) {
  const int ix = t % nx, iy = t / nx;
  const int side = s / m, k = s - side * m;
  const int nv = (nx + 1) * ny;
  int e;
  if (side == 0) {
    e = ix + (nx + 1) * iy;
    dir = ix == 0;
  } else if (side == 1) {
    e = ix + 1 + (nx + 1) * iy;
    dir = ix + 1 == nx;
  } else if (side == 2) {
    e = nv + ix + nx * iy;
    dir = iy == 0;
  } else {
    e = nv + ix + nx * (iy + 1);
    dir = iy + 1 == ny;
  }
  return e * m + k;
}

__device__ __forceinline__ d4 mma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ const double *child_T(const Front &f, bool first, const double *ar,
                                                 const double *S, int nb) {
  const long long o = first ? f.ca : f.cc;
  return o < 0 ? S + (size_t)(-o - 1) * nb * nb : ar + o;
}

// ---------------------------------------------------------------------------
// assembly of the fronts of one level: F = T_a (+) T_c
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_nd_front(const Front *fr, int first, double *ar,
                                                  const int *ia, const double *S, int nb) {
  const Front f = fr[first + blockIdx.y];
  const int nS = f.nS, nE = f.nE, n = nS + nE;
  const long long tot = (long long)n * n;
  const double *Ta = child_T(f, true, ar, S, nb);
  const double *Tc = child_T(f, false, ar, S, nb);
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
// LU with partial pivoting of F_ss, one front per workgroup.  Right-looking
// over 16-column panels: the panel is factored in LDS (largest magnitude in
// the column, ties to the lowest row, as LAPACK getrf), its row exchanges
// are applied to the other columns, U12 = L11^{-1} A12, and the trailing
// block is updated with FP64 MFMA in strips of 16 x 64.  The final row order
// is written to `perm` (row i of P F_ss is row perm[i] of F_ss).
// ---------------------------------------------------------------------------
size_t getrf_lds(int n) {
  const int n16 = (n + 15) & ~15;
  const int nw = kFactorThreads / 64;
  return sizeof(double) * ((size_t)n16 * 16 + nw) + sizeof(int) * (nw + 16 + (size_t)n + 1);
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
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int i = tid; i < n; i += NT) perm[i] = i;
  if (tid == 0) *zp = 0;
  __syncthreads();
  for (int c0 = 0; c0 < n; c0 += 16) {
    const int w = min(16, n - c0), rows = n - c0;
    for (int e = tid; e < rows * 16; e += NT) {
      const int r = e >> 4, c = e & 15;
      P[e] = c < w ? A[(size_t)(c0 + r) * n + c0 + c] : 0.0;
    }
    __syncthreads();
    for (int lc = 0; lc < w; ++lc) {
      double bv = -1.0;
      int br = INT_MAX;
      for (int r = lc + tid; r < rows; r += NT) {
        const double a = fabs(P[r * 16 + lc]);
        if (a > bv) {
          bv = a;
          br = r;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int orow = __shfl_xor(br, off);
        if (ov > bv || (ov == bv && orow < br)) {
          bv = ov;
          br = orow;
        }
      }
      if (lane == 0) {
        redv[wv] = bv;
        redi[wv] = br;
      }
      __syncthreads();
      double pv = redv[0];
      int pr = redi[0];
      for (int k = 1; k < NW; ++k) {
        if (redv[k] > pv || (redv[k] == pv && redi[k] < pr)) {
          pv = redv[k];
          pr = redi[k];
        }
      }
      // no candidate (the whole column NaN): keep the row, flag the pivot
      if (pr >= rows) pr = lc;
      if (pr != lc && tid < 16) {
        const double a = P[lc * 16 + tid];
        P[lc * 16 + tid] = P[pr * 16 + tid];
        P[pr * 16 + tid] = a;
      }
      if (tid == 0) {
        pivl[lc] = c0 + pr;
        if (pr != lc) {
          const int a = perm[c0 + lc];
          perm[c0 + lc] = perm[c0 + pr];
          perm[c0 + pr] = a;
        }
        if (!(pv > 0.0) && *zp == 0) *zp = c0 + lc + 1;
      }
      __syncthreads();
      const double d = P[lc * 16 + lc];
      if (d != 0.0) {
        const double inv = 1.0 / d;
        for (int r = lc + 1 + tid; r < rows; r += NT) {
          const double l = P[r * 16 + lc] * inv;
          P[r * 16 + lc] = l;
          for (int j = lc + 1; j < w; ++j) P[r * 16 + j] -= l * P[lc * 16 + j];
        }
      }
      __syncthreads();
    }
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
    if (c0 + 16 >= n) break;   // last panel: nothing to the right
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
      for (int s = (klo >> 2) + wv; s < (khi >> 2); s += NW) {
        const int kk = 4 * s + (lane >> 4);
        const double a = (arow < n && kk < n) ? A[(size_t)arow * n + kk] : 0.0;
        acc = mma(a, Bs[kk * 16 + (lane & 15)], acc);
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
// r_t = -(w_t + S_t[:, D] g_D) at every slot of every leaf (the Dirichlet
// slots' own entries are never read)
__global__ void k_nd_leaf_rhs(int L, int nx, int ny, int m, const double *S, const double *w,
                              const double *g, double *rl) {
  const int nb = 4 * m;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)L * nb) return;
  const int t = (int)(i / nb), s = (int)(i - (size_t)t * nb);
  bool dir;
  leaf_node(nx, ny, m, t, s, dir);
  double v = w ? w[i] : 0.0;
  if (!dir) {
    const double *row = S + ((size_t)t * nb + s) * nb;
    const double *gt = g + (size_t)t * nb;
    for (int side = 0; side < 4; ++side) {
      bool d;
      leaf_node(nx, ny, m, t, side * m, d);
      if (!d) continue;
      for (int k = side * m; k < side * m + m; ++k) v += row[k] * gt[k];
    }
  }
  rl[i] = dir ? 0.0 : -v;
}


__device__ __forceinline__ const double *child_r(const Front &f, bool first, const double *ar,
                                                 const double *rl, int nb) {
  const long long o = first ? f.ra : f.rc;
  return o < 0 ? rl + (size_t)(-o - 1) * nb : ar + o;
}

// y = r_s and r_b = r_e, scattered from the halves' reduced right-hand sides
__global__ __launch_bounds__(256) void k_nd_front_rhs(const Front *fr, int first, double *ar,
                                                      const int *ia, const double *rl, int nb) {
  const Front f = fr[first + blockIdx.x];
  const int n = f.nS + f.nE;
  const double *ra = child_r(f, true, ar, rl, nb);
  const double *rc = child_r(f, false, ar, rl, nb);
  const int *ma = ia + f.map, *mc = ma + n;
  for (int i = threadIdx.x; i < n; i += 256) {
    double v = 0.0;
    if (ma[i] >= 0) v = ra[ma[i]];
    if (mc[i] >= 0) v += rc[mc[i]];
    if (i < f.nS) ar[f.y + i] = v;
    else ar[f.r + (i - f.nS)] = v;
  }
}

// r_b -= F_es y, one wavefront per row
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
__global__ void k_nd_output(int L, int nx, int ny, int m, const double *u, const double *g,
                            double *ub) {
  const int nb = 4 * m;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)L * nb) return;
  const int t = (int)(i / nb), s = (int)(i - (size_t)t * nb);
  bool dir;
  const int node = leaf_node(nx, ny, m, t, s, dir);
  ub[i] = dir ? g[i] : u[node];
}

// ---------------------------------------------------------------------------
// host planning
// ---------------------------------------------------------------------------
struct Plan {
  int p = 0, m = 0, nb = 0, nx = 0, ny = 0, L = 0;
  std::vector<Front> fronts;      // ordered by level
  std::vector<int> level_first;   // fronts of level l: [level_first[l], level_first[l+1])
  std::vector<int> level_max_s, level_max_e;
  std::vector<int> ints;          // int arena (maps, node ids; pivot orders left 0)
  size_t ndouble = 0;
  int max_sep = 0;
  double flop = 0.0;
  int nnode = 0;                  // edge nodes of the grid (Dirichlet included)
};

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
  int nx, ny, m;
  std::vector<FrontH> fronts;
  int max_sep = 0;

  BoxOut build(int x0, int x1, int y0, int y1) {
    BoxOut out;
    if (x1 - x0 == 1 && y1 - y0 == 1) {
      out.leaf = x0 + nx * y0;
      for (int s = 0; s < 4 * m; ++s) {
        bool dir;
        const int node = leaf_node(nx, ny, m, out.leaf, s, dir);
        if (dir) continue;
        out.E.push_back(node);
        out.pos.push_back(s);
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

hps_status make_plan(int p, int nx, int ny, Plan &pl) {
  if (p < HPS_P_MIN || p > HPS_P_MAX || nx < 1 || ny < 1) return HPS_ERR_INVALID;
  if ((long long)nx * ny > (1 << 22)) return HPS_ERR_INVALID;
  pl.p = p;
  pl.m = p - 2;
  pl.nb = 4 * pl.m;
  pl.nx = nx;
  pl.ny = ny;
  pl.L = nx * ny;
  pl.nnode = ((nx + 1) * ny + nx * (ny + 1)) * pl.m;
  Planner P{nx, ny, pl.m, {}, 0};
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
  auto align = [](size_t v) { return (v + 31) & ~(size_t)31; };
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
    f.fss = (long long)od; od = align(od + s * s);
    f.x = (long long)od;   od = align(od + s * e);
    f.fes = (long long)od; od = align(od + e * s);
    f.t = (long long)od;   od = align(od + e * e);
    f.y = (long long)od;   od = align(od + s);
    f.r = (long long)od;   od = align(od + e);
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
  // children: leaves by code, fronts by their (reordered) arena offsets
  for (int k = 0; k < nf; ++k) {
    const FrontH &h = P.fronts[order[k]];
    Front &f = pl.fronts[k];
    auto child = [&](int c, long long &tOff, long long &rOff, int &ld) {
      if (c < 0) {
        tOff = c;
        rOff = c;
        ld = pl.nb;
      } else {
        const Front &cf = pl.fronts[where[c]];
        tOff = cf.t;
        rOff = cf.r;
        ld = cf.nE;
      }
    };
    child(h.childA, f.ca, f.ra, f.lda);
    child(h.childC, f.cc, f.rc, f.ldc);
  }
  pl.ndouble = od;
  return HPS_OK;
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
  double *d_ar = nullptr;
  int *d_ia = nullptr;
  int *d_info = nullptr;
  double *d_rl = nullptr;   // leaf right-hand sides [L][nb]
  double *d_u = nullptr;    // every edge node's value
};

extern "C" {

hps_status hps_iface_plan(int p, int nx, int ny, int *nfront, int *levels, int *max_sep,
                          double *factor_flop, size_t *bytes) {
  Plan pl;
  try {
    const hps_status st = make_plan(p, nx, ny, pl);
    if (st != HPS_OK) return st;
  } catch (...) {
    return HPS_ERR_OOM;
  }
  if (nfront) *nfront = (int)pl.fronts.size();
  if (levels) *levels = (int)pl.level_first.size() - 2;
  if (max_sep) *max_sep = pl.max_sep;
  if (factor_flop) *factor_flop = pl.flop;
  if (bytes)
    *bytes = pl.ndouble * sizeof(double) + pl.ints.size() * sizeof(int) +
             pl.fronts.size() * (sizeof(Front) + sizeof(int)) +
             ((size_t)pl.L * pl.nb + pl.nnode) * sizeof(double);
  return HPS_OK;
}

hps_status hps_iface_plan_fronts(int p, int nx, int ny, int *nS, int *nE, int *level) {
  Plan pl;
  try {
    const hps_status st = make_plan(p, nx, ny, pl);
    if (st != HPS_OK) return st;
  } catch (...) {
    return HPS_ERR_OOM;
  }
  const int nlev = (int)pl.level_first.size() - 2;
  for (int l = 1; l <= nlev; ++l)
    for (int k = pl.level_first[l]; k < pl.level_first[l + 1]; ++k) {
      if (nS) nS[k] = pl.fronts[k].nS;
      if (nE) nE[k] = pl.fronts[k].nE;
      if (level) level[k] = l;
    }
  return HPS_OK;
}

hps_status hps_iface_create(hps_ctx *ctx, int p, int nx, int ny, hps_iface **out) {
  if (!ctx || !out) return HPS_ERR_INVALID;
  *out = nullptr;
  hps_iface *it = new (std::nothrow) hps_iface;
  if (!it) return HPS_ERR_OOM;
  try {
    const hps_status st = make_plan(p, nx, ny, it->plan);
    if (st != HPS_OK) {
      delete it;
      return st;
    }
  } catch (...) {
    delete it;
    return HPS_ERR_OOM;
  }
  it->stream = hps::ctx_stream(ctx);
  const Plan &pl = it->plan;
  const size_t nf = pl.fronts.size();
  hipError_t e = hipSuccess;
  auto alloc = [&](void **ptr, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMalloc(ptr, bytes);
  };
  alloc((void **)&it->d_front, nf * sizeof(Front));
  alloc((void **)&it->d_ar, pl.ndouble * sizeof(double));
  alloc((void **)&it->d_ia, pl.ints.size() * sizeof(int));
  alloc((void **)&it->d_info, (nf + 1) * sizeof(int));
  alloc((void **)&it->d_rl, (size_t)pl.L * pl.nb * sizeof(double));
  alloc((void **)&it->d_u, (size_t)pl.nnode * sizeof(double));
  if (e == hipSuccess && nf)
    e = hipMemcpy(it->d_front, pl.fronts.data(), nf * sizeof(Front), hipMemcpyHostToDevice);
  if (e == hipSuccess && !pl.ints.empty())
    e = hipMemcpy(it->d_ia, pl.ints.data(), pl.ints.size() * sizeof(int),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess) e = allow_lds(k_nd_getrf, getrf_lds(kMaxSep));
  if (e == hipSuccess) e = allow_lds(k_nd_getrs, getrs_lds(kMaxSep));
  if (e != hipSuccess) {
    hps_iface_destroy(it);
    return from_hip(e);
  }
  *out = it;
  return HPS_OK;
}

hps_status hps_iface_factor(hps_iface *it, const double *S, int *info, int flags) {
  if (!it || !S) return HPS_ERR_INVALID;
  const Plan &pl = it->plan;
  const hipStream_t st = it->stream;
  const int nlev = (int)pl.level_first.size() - 2;
  for (int l = 1; l <= nlev; ++l) {
    const int first = pl.level_first[l], cnt = pl.level_first[l + 1] - first;
    if (cnt <= 0) continue;
    const int ms = pl.level_max_s[l], me = pl.level_max_e[l];
    const long long nn = (long long)(ms + me) * (ms + me);
    const int gx = (int)std::min<long long>((nn + 255) / 256, 4096);
    k_nd_front<<<dim3(gx, cnt), 256, 0, st>>>(it->d_front, first, it->d_ar, it->d_ia, S, pl.nb);
    k_nd_getrf<<<cnt, kFactorThreads, getrf_lds(ms), st>>>(it->d_front, first, it->d_ar,
                                                            it->d_ia, it->d_info);
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
  const size_t nslot = (size_t)pl.L * pl.nb;
  const int gs = (int)((nslot + 255) / 256);
  k_nd_leaf_rhs<<<gs, 256, 0, st>>>(pl.L, pl.nx, pl.ny, pl.m, S, w, g, it->d_rl);
  for (int l = 1; l <= nlev; ++l) {
    const int first = pl.level_first[l], cnt = pl.level_first[l + 1] - first;
    if (cnt <= 0) continue;
    const int ms = pl.level_max_s[l], me = pl.level_max_e[l];
    k_nd_front_rhs<<<cnt, 256, 0, st>>>(it->d_front, first, it->d_ar, it->d_ia, it->d_rl,
                                        pl.nb);
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
  k_nd_output<<<gs, 256, 0, st>>>(pl.L, pl.nx, pl.ny, pl.m, it->d_u, g, ub);
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
  rel(it->d_ar);
  rel(it->d_ia);
  rel(it->d_info);
  rel(it->d_rl);
  rel(it->d_u);
  delete it;
  return from_hip(first);
}

}  // extern "C"
