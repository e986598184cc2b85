// Host-side multigrid hierarchy produced by the setup and consumed by the
// device upload. Plain C++17; no HIP types.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

namespace vasmg {

// Setup failure: status is a vasmg_status value.
struct Error {
  int status;
  std::string msg;
};

using Key = std::array<uint64_t, 3>;   // lattice key per axis (unused axes 0)

// d x d block CSR, structural pattern including the diagonal block, columns
// ascending within a row. val holds row-major d x d blocks.
struct BlockCSR {
  int64_t n = 0;
  int d = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  int64_t nnzb() const { return static_cast<int64_t>(col.size()); }
};

// Scalar CSR (prolongation weights; the same weight applies to every component).
struct ScalarCSR {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

struct Level {
  int64_t n = 0;               // vertices
  std::vector<Key> keys;       // coarse levels: lattice keys in canonical order
  BlockCSR A;                  // operator, canonical vertex order
  int max_region_depth = 0;    // coarse levels: deepest region of the level
  // Gauss-Seidel order (levels below the coarsest): vertex -> cell, cell -> colour
  std::vector<int32_t> cell;
  std::vector<int32_t> cell_color;
  int64_t ncells = 0;
  std::vector<int32_t> color;  // colour of each vertex's cell
  int32_t ncolors = 0;
  ScalarCSR P;                 // prolongation to the next level (empty on the coarsest)
};

struct Hierarchy {
  int d = 0;
  int64_t n_mesh_vertices = 0;
  std::vector<int32_t> free_vertices;   // fine canonical order -> mesh vertex
  std::vector<Level> levels;            // levels[0] = fine, levels.back() = coarsest
  std::vector<double> chol;             // lower Cholesky factor of the coarsest, row-major
  int64_t n_coarse_dofs = 0;
  double box_m = 0.0, box_M = 0.0;      // root box [m, M]^d
  int max_depth = 0;
  int capacity = 0;
  // wall-clock milliseconds of the setup phases, in the order they ran
  std::vector<std::pair<std::string, double>> phase_ms;
};

struct MeshView {
  int d;
  int64_t nv;
  const double* coords;
  int64_t ne;
  const int32_t* elems;
  const double* E;
  const double* nu;
  const uint8_t* fixed;
};

// Galerkin product A_c = P^T A P (block A, scalar P shared by the components).
using GalerkinFn = void (*)(void* ctx, const BlockCSR& A, const ScalarCSR& P, BlockCSR& Ac);

struct SetupParams {
  int capacity;                // leaf capacity (> 0)
  bool tree_free_only;         // tree over free vertices only
  int64_t coarsest_max_dofs;   // 0 = root level
  GalerkinFn galerkin = nullptr;   // null: the host product (OpenMP)
  void* galerkin_ctx = nullptr;
};

// Device Galerkin products (galerkin.hip): a context with its own stream that
// keeps the last coarse operator resident as the next product's A.
// window_cols > 0 caps the columns per symbolic pass (0 = the LDS maximum).
struct GalerkinDevice;
GalerkinDevice* galerkin_device_create(int window_cols);
void galerkin_device_destroy(GalerkinDevice* g);
void galerkin_device(void* ctx, const BlockCSR& A, const ScalarCSR& P, BlockCSR& Ac);

// Builds the whole hierarchy on the host. Throws vasmg::Error.
void build_hierarchy(const MeshView& mesh, const SetupParams& prm, Hierarchy& out);

// Damped vertex-block Jacobi smoother data: inverse diagonal blocks [n][d][d]
// (canonical order) and the largest eigenvalue of D^{-1} A by power iteration.
void block_diag_inverse(const BlockCSR& A, std::vector<double>& out);
double jacobi_lambda_max(const BlockCSR& A, const std::vector<double>& dinv, int iters);

}  // namespace vasmg
