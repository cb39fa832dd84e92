// GMRES workspace and kernel launchers (device resident, float64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ibim {

struct Krylov {
  int m = 0;               // restart length
  int64_t n = 0;           // vector length (2M)
  double* V = nullptr;     // (m+1) * n, column c at V + c*n
  double* H = nullptr;     // (m+1) * m row-major
  double* cs = nullptr;    // m
  double* sn = nullptr;    // m
  double* g = nullptr;     // m+1
  double* y = nullptr;     // m
  double* hcol = nullptr;  // m+1 Gram-Schmidt coefficients of the current column
  double* hcol2 = nullptr; // m+1 second-pass coefficients
  double* scal = nullptr;  // 4 device scalars (squared norms)
  double* status = nullptr;// 2 device scalars: |g_{j+1}|, H(j+1, j)
  double* partial = nullptr;  // (m+1) * 1024 reduction scratch
  double* tmp = nullptr;   // n: residual / scratch vector
  double* tmp2 = nullptr;  // n: scratch vector
  double* bsc = nullptr;   // n: right-hand side of the row-scaled system
  double* host_status = nullptr;  // pinned host mirror of status

  static int dot_blocks(int64_t n);
  hipError_t dots(const double* V, int64_t ldv, int ncols, const double* w, int64_t n, double* out,
                  int accumulate, hipStream_t s);
  hipError_t sub(const double* V, int64_t ldv, int ncols, const double* coef, double* w, int64_t n,
                 hipStream_t s);
  hipError_t add(const double* V, int64_t ldv, int ncols, const double* coef, double* x, int64_t n,
                 hipStream_t s);
  hipError_t normalize(const double* x, const double* nrm2, double* y, int64_t n, hipStream_t s);
  hipError_t residual(const double* b, const double* Ax, double* r, int64_t n, hipStream_t s);
  hipError_t givens(int j, hipStream_t s);
  hipError_t init_g(const double* nrm2, hipStream_t s);
  hipError_t backsolve(int n, hipStream_t s);
};

// One Arnoldi + Givens step of many independent solves, one launch per stage
// for all of them: solve q orthogonalises w = V_{j+1} (holding A V_j on
// entry) against V_0..V_j twice (classical Gram-Schmidt, as the single-solve
// sequence dots/sub/dots/sub), normalises it and applies the Givens step.
// Every solve gets exactly the blocks and reduction order of the
// single-solve launchers, so its bits do not depend on the batch.
struct KrylovStepArgs {
  const double* V;  // basis of the solve; w = V + (j + 1) n
  double *H, *cs, *sn, *g, *hcol, *hcol2, *scal, *partial;  // its Krylov workspace
  double* status;   // out: |g_{j+1}|, H(j+1, j)
  int64_t n;
  int m, j;
  // filled by krylov_step_batched: dot-product blocks of n, and this solve's
  // first block in the launches over V (nblk (j+1) blocks), over w alone
  // (nblk), the reductions (j + 1) and the row launches (ceil(n / 256))
  int nblk, rows_per;
  int64_t dot0, dotw0, red0, vec0;
};

// steps: pinned host array of count entries (the block fields are filled
// here); d_steps: device array of count entries, written on stream s from
// steps, which must stay unchanged until s has passed this point.
hipError_t krylov_step_batched(KrylovStepArgs* steps, int count, KrylovStepArgs* d_steps,
                               hipStream_t s);

}  // namespace ibim
