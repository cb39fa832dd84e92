// Internal declarations shared by the library's host and device sources.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ibim {

constexpr double kPi = 3.14159265358979323846;

// Result of the host part of the setup (geometry + correction sets).
struct HostPlan {
  int64_t M = 0;
  int dims[3] = {0, 0, 0};
  double origin[3] = {0, 0, 0};
  double h = 0, eps = 0;
  std::vector<int64_t> grid_index;  // M: linear grid index of each node
  // node geometry, structure of arrays
  std::vector<double> px, py, pz;   // projection P(y)
  std::vector<double> nx, ny, nz;   // outward unit normal
  std::vector<double> w;            // J * delta_eps(d)
  std::vector<double> kap1, kap2;   // surface principal curvatures at P(y)
  std::vector<double> tau;          // 6M: principal directions tau1 (0..2), tau2 (3..5)
  // correction sets, CSR sorted by column within each row
  std::vector<int64_t> crow;        // M+1
  std::vector<int32_t> ccol;        // nnz
  std::vector<int32_t> crowid;      // nnz: owning row
  std::vector<int8_t> caxis;        // nnz: dominant axis of the row; -1: K-reg entry
  std::vector<double> calpha, cbeta, ceta;
  // HYB-IBIM: nodes in M_B (K-reg rows, J = 1) and the K-reg constant of K12
  std::vector<uint8_t> bad;         // M
  double ktau = 0.0;                // K-reg radius (2h)
  int64_t n_bad = 0;
};

// OpenMP threads used by build_host_plan when called from the current host
// thread (setup threads of the solve server share the cores).
void set_host_setup_threads(int n);

// Builds the plan; returns 0 or a negative IBIM_E* code with *err set.
// hybrid: 0 CTR2 rows everywhere, 1 HYB-IBIM, 2 every node bad (K-reg).
int build_host_plan(const double* sdf, int nx, int ny, int nz, const double origin[3], double h,
                    double eps, int hybrid, HostPlan* plan, std::string* err);

}  // namespace ibim
