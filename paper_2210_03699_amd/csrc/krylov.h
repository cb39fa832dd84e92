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

}  // namespace ibim
