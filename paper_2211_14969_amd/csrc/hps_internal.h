// Internal declarations shared by the HIP kernels and the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

struct hps_ctx;

namespace hps {

// The stream a context enqueues on (hps_abi.hip).
hipStream_t ctx_stream(const ::hps_ctx *c);

// One order-p group of leaves as the kernels see it (pointers already offset
// to the first leaf of the launch).
struct Geom {
  int p;        // points per direction
  int m;        // p - 2
  int ni;       // (p-2)^2 interior nodes
  int nb;       // 4(p-2) edge nodes
  int R;        // ni rounded up to 16: rows / A-part columns of the work matrix
  int RT;       // R / 16 row tiles
  int CT;       // column tiles of the work matrix (A part + right-hand sides)
  int mdiv;     // ceil(2^16 / m): n / m == (n * mdiv) >> 16 for 0 <= n < 2048
  int nrhs;     // right-hand-side columns in use
  const double *box;                        // [nleaf][4]
  const double *a11, *a22, *c1, *c2, *k2b;  // [nleaf][p*p] or nullptr
  const double *a12;                        // [nleaf][p*p] or nullptr (mixed term)
  const double *D;                          // [p][p]  d/dt on [-1, 1]
  const double *D2;                         // [p][p]  D*D
  const double *E;                          // [2][p-2] corner extrapolation weights
  int tune_variant;   // factorisation: 0 automatic, 1 one panel per pass, 2 panel pairs,
                      // 3 register-resident (FP32, R <= 208)
  int tune_ch;        // column chunk of the U12 / trailing passes (0 automatic)
};

// 16 x 16 tiles of one leaf's slot in the factorisation workspace: the work
// matrix (RT x CT tiles) and one tile per panel for its L11^{-1}.
__host__ __device__ inline size_t leaf_tiles(const Geom &g) {
  return (size_t)g.RT * (g.CT + 1);
}

// Right-hand-side layouts of the work matrix.
enum RhsMode : int {
  RHS_CONDENSE = 0,  // columns: A_ib (nb), then f_i if present
  RHS_REFACTOR = 1   // one column: f_i - A_ib u_b
};

// Where the back substitution puts its result.
enum BackMode : int {
  BACK_STORE = 0,    // X -> Xt (FP64, transposed), h -> h
  BACK_ACCUM = 1,    // Xt += dX, h += dh
  BACK_UI = 2        // single column -> ui
};

// Leaf selection of a launch: block b uses work-matrix slot b and, when
// `list` is set, leaf list[slot0 + b]; blocks at or past *count exit at once.
struct Sel {
  const int *list = nullptr;
  const int *count = nullptr;
  int slot0 = 0;
};

struct BackOut {
  double *Xt;        // [nleaf][nb][ni]
  double *h;         // [nleaf][ni]   (nullptr when no f column)
  double *ui;        // [nleaf][ni]   (BACK_UI)
  double *norms;     // [nleaf][kNormStride]: slot 16 + chunk receives ||dX||^2 (BACK_ACCUM)
  const int *skip;   // [nleaf] leaves to leave untouched (nullptr = none)
  int mode;
};

constexpr int kInfoActive = 0x7fffffff;
// refinement norms per leaf: 0 ||r||^2, 1 ||X||^2, 4 previous ||r||^2,
// 5 ||dX||^2 of the last correction, 6 relative size of the first correction;
// per column chunk c < kMaxChunks: 8+c ||r||^2, 12+c ||X||^2 (residual) and
// 16+c ||dX||^2 (correction), summed in chunk order by the stop test
constexpr int kMaxChunks = 4;
constexpr int kNormStride = 24;

// Launchers (hps_kernels.hip).  All enqueue on `s` and return hipError_t.
// Factorisation of the work matrices; step 0 forms them from the operator
// (mode RHS_CONDENSE with optional f, or RHS_REFACTOR with f and ub).
hipError_t launch_factor(const Geom &g, int nleaf, bool fp32, void *M, int *piv,
                         int *rstep, int *info, int mode, const double *f, const double *ub,
                         hipStream_t s, const Sel &sel = Sel());
hipError_t launch_backsolve(const Geom &g, int nleaf, bool fp32, void *M,
                            const int *piv, const int *rstep, const BackOut &o,
                            hipStream_t s, const Sel &sel = Sel());
// forward + back substitution of FP32 factors on the right-hand sides held in
// the work matrix (the refinement residual), accumulating into o.Xt / o.h
hipError_t launch_refine_solve(const Geom &g, int nleaf, void *M, const int *piv,
                               const int *rstep, const BackOut &o, int nch, hipStream_t s);
hipError_t launch_residual(const Geom &g, int nleaf, float *M32, const double *Xt,
                           const double *h, const double *f, const int *skip,
                           double *norms, int nch, hipStream_t s);
hipError_t launch_convcheck(int nleaf, double *norms, double tol, int *conv, int *info,
                            int it, int last, int nres, int nsol, hipStream_t s);
// column chunks (workgroups per leaf) of the refinement residual and
// correction solve; more than one only for iterations after the first,
// where the few leaves left would otherwise leave the GPU idle
int refine_chunks(const Geom &g, int it);
// norm slots the correction solve of that many chunks writes (the
// register-resident solves split by their own column chunks)
int refine_solve_chunks(const Geom &g, int nch);
hipError_t launch_collect(int nleaf, int *info, int *list, int *count, int *total, int *redo,
                          hipStream_t s);
hipError_t launch_schur(const Geom &g, int nleaf, const double *Xt, const double *h,
                        double *S, double *w, int *info, hipStream_t s);
hipError_t launch_recover(const Geom &g, int nleaf, const double *Xt, const double *h,
                          const double *ub, double *ui, hipStream_t s);
hipError_t launch_operator(const Geom &g, int nleaf, double *Aii, double *Aib,
                           double *Abi, double *Abb, hipStream_t s);
hipError_t launch_nodes(const Geom &g, int nleaf, const double *t, double *xy,
                        hipStream_t s);
hipError_t launch_fill_int(int *dst, int n, int v, hipStream_t s);
hipError_t launch_fill_double(double *dst, size_t n, double v, hipStream_t s);
hipError_t launch_copy_info(const int *src, int *dst, int n, hipStream_t s);

// Bytes of dynamic LDS the factor kernel needs; 0 if it does not fit.
size_t factor_lds_bytes(const Geom &g, bool fp32);

// Host tables (hps_cheb.cpp).
// t [p], D [p*p], D2 [p*p], E [2][p-2]; cheb_table_size(p) doubles in all.
void cheb_tables(int p, double *t, double *D, double *D2, double *E);
inline size_t cheb_table_size(int p) { return (size_t)p + 2 * (size_t)p * p + 2 * (size_t)(p - 2); }

}  // namespace hps
