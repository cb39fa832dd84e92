// Device construction of the CTR2 correction weights and blocks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ibim {

constexpr double kPiD = 3.14159265358979323846;

struct WeightArgs {
  int64_t nnz;
  const int32_t* rowid;  // nnz: target row of each entry
  const int32_t* col;    // nnz: corrected node
  const int8_t* axis;    // nnz: dominant axis of the row
  const double* alpha;   // nnz
  const double* beta;    // nnz
  const double* eta;     // nnz
  const double* tau;     // 6M principal directions
  const double* kap1;    // M
  const double* kap2;    // M
  const double* w;       // M
  double eps_in, eps_out, kappa, h;
  double c12;            // K-reg constant of K12 (entries with axis -1)
  double* om11;          // nnz out: omega[s0^(11)]
  double* om21;          // nnz out: omega[s0^(21)]
  double* blocks;        // 4*nnz out: the 2x2 block of h^2 Omega W per entry
};

hipError_t launch_weights(const WeightArgs& a, hipStream_t stream);

// Mean of K12 over the tangent disc of radius tau (the K-reg constant of
// eq. regularized-kernel): (e^{-k tau} - 1 + k tau) / (2 pi k tau^2).
double kreg_constant(double kappa, double tau);

}  // namespace ibim
