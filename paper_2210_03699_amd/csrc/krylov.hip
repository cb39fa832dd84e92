// Device kernels of the GMRES solve (Section 2.5): block dot products with a
// fixed-order two-pass reduction (deterministic), vector updates for
// classical Gram-Schmidt with one re-orthogonalisation, and single-lane
// kernels for the Givens rotations and the triangular solve.  All float64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "krylov.h"

namespace ibim {
namespace {

constexpr int kDotThreads = 256;

// partial[c * nblk + b] = sum over rows of block b of V_c . w (one block)
__device__ __forceinline__ void dots_block(const double* V, int64_t ldv, const double* w, int64_t n,
                                           int rows_per, int c, int b, int nblk, double* partial,
                                           double* red) {
  const double* v = V + (int64_t)c * ldv;
  const int64_t r0 = (int64_t)b * rows_per;
  const int64_t r1 = r0 + rows_per < n ? r0 + rows_per : n;
  double acc = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += kDotThreads) acc += v[r] * w[r];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kDotThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)c * nblk + b] = red[0];
}

__global__ __launch_bounds__(kDotThreads) void dots_kernel(const double* V, int64_t ldv, int ncols,
                                                           const double* w, int64_t n, int rows_per,
                                                           double* partial) {
  __shared__ double red[kDotThreads];
  dots_block(V, ldv, w, n, rows_per, blockIdx.y, blockIdx.x, gridDim.x, partial, red);
  (void)ncols;
}

// out[c] = sum_b partial[c * nblk + b] (+ out[c] if accumulate) (one block)
__device__ __forceinline__ void reduce_block(const double* partial, int nblk, int c, double* out,
                                             int accumulate, double* red) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kDotThreads) acc += partial[(int64_t)c * nblk + b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kDotThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = accumulate ? out[c] + red[0] : red[0];
}

__global__ __launch_bounds__(kDotThreads) void reduce_kernel(const double* partial, int nblk,
                                                             double* out, int accumulate) {
  __shared__ double red[kDotThreads];
  reduce_block(partial, nblk, blockIdx.x, out, accumulate, red);
}

// w -= sum_c coef[c] V_c (row r)
__device__ __forceinline__ void sub_row(const double* V, int64_t ldv, int ncols,
                                        const double* coef, double* w, int64_t r) {
  double acc = w[r];
  for (int c = 0; c < ncols; ++c) acc -= coef[c] * V[(int64_t)c * ldv + r];
  w[r] = acc;
}

__global__ __launch_bounds__(256) void sub_kernel(const double* V, int64_t ldv, int ncols,
                                                  const double* coef, double* w, int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  sub_row(V, ldv, ncols, coef, w, r);
}

// x += sum_c coef[c] V_c
__global__ __launch_bounds__(256) void add_kernel(const double* V, int64_t ldv, int ncols,
                                                  const double* coef, double* x, int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double acc = x[r];
  for (int c = 0; c < ncols; ++c) acc += coef[c] * V[(int64_t)c * ldv + r];
  x[r] = acc;
}

// y = x / sqrt(*nrm2)
__global__ __launch_bounds__(256) void scale_kernel(const double* x, const double* nrm2, double* y,
                                                    int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double inv = 1.0 / sqrt(*nrm2);
  y[r] = x[r] * inv;
}

// y = b - x
__global__ __launch_bounds__(256) void axpby_kernel(const double* b, const double* x, double* y,
                                                    int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  y[r] = b[r] - x[r];
}

// One Givens step on Hessenberg column j (single lane).
// H is (m+1) x m row-major (H[i*m + j]); hcol and hcol2 hold the two
// Gram-Schmidt passes' coefficients of column j, *wn2 the squared norm of
// the orthogonalised w.
__device__ __forceinline__ void givens_lane(double* H, int m, int j, const double* hcol,
                                            const double* hcol2, const double* wn2, double* cs,
                                            double* sn, double* g, double* status) {
  for (int i = 0; i <= j; ++i) H[i * m + j] = hcol[i] + hcol2[i];
  const double hn = sqrt(*wn2);
  H[(j + 1) * m + j] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = H[i * m + j], b = H[(i + 1) * m + j];
    H[i * m + j] = cs[i] * a + sn[i] * b;
    H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
  }
  const double a = H[j * m + j], b = H[(j + 1) * m + j];
  const double den = hypot(a, b);
  cs[j] = a / den;
  sn[j] = b / den;
  H[j * m + j] = den;
  H[(j + 1) * m + j] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  status[0] = fabs(g[j + 1]);
  status[1] = hn;
}

__global__ void givens_kernel(double* H, int m, int j, const double* hcol, const double* hcol2,
                              const double* wn2, double* cs, double* sn, double* g,
                              double* status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  givens_lane(H, m, j, hcol, hcol2, wn2, cs, sn, g, status);
}

// Back substitution H(0:n,0:n) y = g (single lane).
__global__ void backsolve_kernel(const double* H, int m, int n, const double* g, double* y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = n - 1; i >= 0; --i) {
    double s = g[i];
    for (int t = i + 1; t < n; ++t) s -= H[i * m + t] * y[t];
    y[i] = s / H[i * m + i];
  }
}

__global__ void init_g_kernel(double* g, int m, const double* nrm2) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = 0; i <= m; ++i) g[i] = 0.0;
  g[0] = sqrt(*nrm2);
}

inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

// Batched stages.  Field f of the step table: 0 dot0, 1 dotw0, 2 red0, 3 vec0;
// the block's solve is the last one whose first block is <= blk.
__device__ __forceinline__ int64_t first_block(const KrylovStepArgs& a, int f) {
  return f == 0 ? a.dot0 : f == 1 ? a.dotw0 : f == 2 ? a.red0 : a.vec0;
}

__device__ __forceinline__ int find_solve(const KrylovStepArgs* st, int count, int64_t blk, int f) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (first_block(st[mid], f) <= blk) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// which = 0: hcol = V^T w; 1: hcol2 = V^T w; 2: scal = w . w
__global__ __launch_bounds__(kDotThreads) void dots_batched_kernel(const KrylovStepArgs* st,
                                                                   int count, int which) {
  __shared__ double red[kDotThreads];
  const int64_t blk = blockIdx.x;
  const int f = which == 2 ? 1 : 0;
  const KrylovStepArgs& a = st[find_solve(st, count, blk, f)];
  const int64_t loc = blk - first_block(a, f);
  const double* w = a.V + (int64_t)(a.j + 1) * a.n;
  const double* V = which == 2 ? w : a.V;
  dots_block(V, a.n, w, a.n, a.rows_per, (int)(loc / a.nblk), (int)(loc % a.nblk), a.nblk,
             a.partial, red);
}

__global__ __launch_bounds__(kDotThreads) void reduce_batched_kernel(const KrylovStepArgs* st,
                                                                     int count, int which) {
  __shared__ double red[kDotThreads];
  if (which == 2) {  // one reduction per solve
    const KrylovStepArgs& a = st[blockIdx.x];
    reduce_block(a.partial, a.nblk, 0, a.scal, 0, red);
    return;
  }
  const int64_t blk = blockIdx.x;
  const KrylovStepArgs& a = st[find_solve(st, count, blk, 2)];
  reduce_block(a.partial, a.nblk, (int)(blk - a.red0), which == 0 ? a.hcol : a.hcol2, 0, red);
}

// which = 0: w -= V hcol; 1: w -= V hcol2; 2: w /= sqrt(scal)
__global__ __launch_bounds__(256) void rows_batched_kernel(const KrylovStepArgs* st, int count,
                                                           int which) {
  const int64_t blk = blockIdx.x;
  const KrylovStepArgs& a = st[find_solve(st, count, blk, 3)];
  const int64_t r = (blk - a.vec0) * 256 + threadIdx.x;
  if (r >= a.n) return;
  double* w = const_cast<double*>(a.V) + (int64_t)(a.j + 1) * a.n;
  if (which == 2) {
    const double inv = 1.0 / sqrt(*a.scal);
    w[r] = w[r] * inv;
  } else {
    sub_row(a.V, a.n, a.j + 1, which == 0 ? a.hcol : a.hcol2, w, r);
  }
}

__global__ void givens_batched_kernel(const KrylovStepArgs* st) {
  if (threadIdx.x != 0) return;
  const KrylovStepArgs& a = st[blockIdx.x];
  givens_lane(a.H, a.m, a.j, a.hcol, a.hcol2, a.scal, a.cs, a.sn, a.g, a.status);
}

}  // namespace

int Krylov::dot_blocks(int64_t n) {
  // enough blocks to fill the GPU, each a whole multiple of the block size
  int64_t b = (n + 4096 - 1) / 4096;
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

hipError_t Krylov::dots(const double* V, int64_t ldv, int ncols, const double* w, int64_t n,
                        double* out, int accumulate, hipStream_t s) {
  const int nblk = dot_blocks(n);
  const int rows_per = (int)((n + nblk - 1) / nblk);
  hipLaunchKernelGGL(dots_kernel, dim3(nblk, ncols), dim3(kDotThreads), 0, s, V, ldv, ncols, w, n,
                     rows_per, partial);
  hipLaunchKernelGGL(reduce_kernel, dim3(ncols), dim3(kDotThreads), 0, s, partial, nblk, out,
                     accumulate);
  return hipGetLastError();
}

hipError_t Krylov::sub(const double* V, int64_t ldv, int ncols, const double* coef, double* w,
                       int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(sub_kernel, dim3(nb(n)), dim3(256), 0, s, V, ldv, ncols, coef, w, n);
  return hipGetLastError();
}

hipError_t Krylov::add(const double* V, int64_t ldv, int ncols, const double* coef, double* x,
                       int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(add_kernel, dim3(nb(n)), dim3(256), 0, s, V, ldv, ncols, coef, x, n);
  return hipGetLastError();
}

hipError_t Krylov::normalize(const double* x, const double* nrm2, double* y, int64_t n,
                             hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(nb(n)), dim3(256), 0, s, x, nrm2, y, n);
  return hipGetLastError();
}

hipError_t Krylov::residual(const double* b, const double* Ax, double* r, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, dim3(nb(n)), dim3(256), 0, s, b, Ax, r, n);
  return hipGetLastError();
}

hipError_t Krylov::givens(int j, hipStream_t s) {
  hipLaunchKernelGGL(givens_kernel, dim3(1), dim3(64), 0, s, H, m, j, hcol, hcol2, scal, cs, sn,
                     g, status);
  return hipGetLastError();
}

hipError_t Krylov::init_g(const double* nrm2, hipStream_t s) {
  hipLaunchKernelGGL(init_g_kernel, dim3(1), dim3(64), 0, s, g, m, nrm2);
  return hipGetLastError();
}

hipError_t Krylov::backsolve(int n, hipStream_t s) {
  hipLaunchKernelGGL(backsolve_kernel, dim3(1), dim3(64), 0, s, H, m, n, g, y);
  return hipGetLastError();
}

hipError_t krylov_step_batched(KrylovStepArgs* st, int count, KrylovStepArgs* d_st,
                               hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t dot = 0, dotw = 0, red = 0, vec = 0;
  for (int q = 0; q < count; ++q) {
    KrylovStepArgs& a = st[q];
    a.nblk = Krylov::dot_blocks(a.n);
    a.rows_per = (int)((a.n + a.nblk - 1) / a.nblk);
    a.dot0 = dot;
    a.dotw0 = dotw;
    a.red0 = red;
    a.vec0 = vec;
    dot += (int64_t)a.nblk * (a.j + 1);
    dotw += a.nblk;
    red += a.j + 1;
    vec += nb(a.n);
  }
  hipError_t e = hipMemcpyAsync(d_st, st, sizeof(KrylovStepArgs) * (size_t)count,
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  const dim3 t(kDotThreads);
  for (int pass = 0; pass < 2; ++pass) {  // Gram-Schmidt and its re-orthogonalisation
    hipLaunchKernelGGL(dots_batched_kernel, dim3((unsigned)dot), t, 0, s, d_st, count, pass);
    hipLaunchKernelGGL(reduce_batched_kernel, dim3((unsigned)red), t, 0, s, d_st, count, pass);
    hipLaunchKernelGGL(rows_batched_kernel, dim3((unsigned)vec), dim3(256), 0, s, d_st, count,
                       pass);
  }
  hipLaunchKernelGGL(dots_batched_kernel, dim3((unsigned)dotw), t, 0, s, d_st, count, 2);
  hipLaunchKernelGGL(reduce_batched_kernel, dim3((unsigned)count), t, 0, s, d_st, count, 2);
  hipLaunchKernelGGL(rows_batched_kernel, dim3((unsigned)vec), dim3(256), 0, s, d_st, count, 2);
  hipLaunchKernelGGL(givens_batched_kernel, dim3((unsigned)count), dim3(64), 0, s, d_st);
  return hipGetLastError();
}

}  // namespace ibim
