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

// Allocator whose resize() leaves new elements uninitialised (default-init):
// the column arrays of the coarse levels are filled by a copy right after they
// are sized, and zero-filling 10^8 entries first costs tens of milliseconds.
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};
using ColVec = std::vector<int32_t, NoInitAlloc<int32_t>>;

// d x d block CSR, structural pattern including the diagonal block, columns
// ascending within a row. val holds row-major d x d blocks.
struct BlockCSR {
  int64_t n = 0;
  int d = 0;
  std::vector<int64_t> rowptr;
  ColVec col;
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
  // Gauss-Seidel order (levels below the coarsest): vertex -> cell, vertex ->
  // colour block (whole cells), block -> colour. A sweep visits colours, the
  // blocks of a colour, the cells of a block and the vertices of a cell in
  // canonical order. block_steps: side of the blocks in lattice steps (2: a
  // block is one cell; 4: up to 2^d cells; fine level: 1).
  std::vector<int32_t> cell;
  int64_t ncells = 0;
  std::vector<int32_t> block;
  std::vector<int32_t> block_color;
  int64_t nblocks = 0;
  int block_steps = 1;
  std::vector<int32_t> color;  // colour of each vertex's block
  int32_t ncolors = 0;
  ScalarCSR P;                 // prolongation to the next level (empty on the coarsest)
  // Constrained components (homogeneous Dirichlet on some components of a
  // vertex, or coarse components whose interpolating fine vertices all have
  // them fixed): bit a of fixed[i] set = component a of vertex i. Empty when the
  // level has none. A stores zero rows and columns there; the solve operator
  // has an identity row and column (layouts, export, coarsest factor).
  std::vector<uint8_t> fixed;
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
// `coarsest`: A_c is the last level (its values are needed on the host at once).
using GalerkinFn = void (*)(void* ctx, const BlockCSR& A, const ScalarCSR& P, BlockCSR& Ac,
                            bool coarsest);

// Fine-level assembly of A (free vertices in ascending mesh order, vfree: mesh
// vertex -> free index or -1); the structure must be on the host on return.
using AssembleFn = void (*)(void* ctx, const MeshView& m, const std::vector<int32_t>& vfree,
                            int64_t nfree, BlockCSR& A);
// Brings every level's values to the host (values produced elsewhere).
using SettleFn = void (*)(void* ctx);
// Waits until level l's structure (l < 0: every level's) has reached the host
// hierarchy; rethrows a failed download.
using WaitFn = void (*)(void* ctx, int level);

// Region tree, level lattice keys and prolongations (Section 3.1.1 Steps 1-4,
// Section 3.1.2, Section 3.2) built elsewhere with the host build's decisions,
// keys and weights: P[l] prolongs level l + 1 to level l, keys[l] and
// max_region_depth[l] describe level l >= 1 (keys[0] is empty).
struct Transfers {
  double m = 0.0, M = 0.0;   // root box
  int max_depth = 0;
  std::vector<ScalarCSR> P;
  std::vector<std::vector<Key>> keys;
  std::vector<int> max_region_depth;
};
// Returns false (out untouched) where it cannot build them: the host does.
using TransfersFn = bool (*)(void* ctx, const MeshView& m, const std::vector<int32_t>& tree_vtx,
                             const std::vector<int32_t>& free_vertices,
                             const std::vector<int32_t>& pos_in_tree, int capacity, Transfers& out);

struct SetupParams {
  int capacity;                // leaf capacity (> 0)
  bool tree_free_only;         // tree over free vertices only
  int64_t coarsest_max_dofs;   // 0 = root level
  bool color_blocks = false;   // colour blocks of 4 lattice steps where the reach allows (3D)
  GalerkinFn galerkin = nullptr;   // null: the host product (OpenMP)
  AssembleFn assemble = nullptr;   // null: the host assembly (OpenMP)
  SettleFn settle = nullptr;
  WaitFn wait_structure = nullptr;   // null: a product's structure is home on return
  TransfersFn transfers = nullptr;   // null: the host tree and prolongations
  void* galerkin_ctx = nullptr;    // context of the callbacks
};

// Vertex -> element lists (elements ascending per vertex).
void vertex_elements(const MeshView& m, std::vector<int64_t>& vptr, std::vector<int64_t>& velem);

// Device setup (galerkin.hip): a context with its own stream that keeps every
// level's canonical FP64 operator resident (level 0 uploaded, the others the
// products), hands the host each product's structure at once and its values
// from background downloads, and builds the device layout of a level from the
// resident operator. window_cols > 0 caps the columns per symbolic pass of the
// product (0 = the LDS maximum).
struct GalerkinDevice;
GalerkinDevice* galerkin_device_create(int window_cols);
void galerkin_device_destroy(GalerkinDevice* g);   // joins the downloads
void galerkin_device(void* ctx, const BlockCSR& A, const ScalarCSR& P, BlockCSR& Ac,
                     bool coarsest);
// Fine-level assembly on the device (the same element order and arithmetic as
// the host assembly, so the same values bit for bit): the structure comes back
// at once, the values stay resident as level 0 and download in the background.
void assemble_device(void* ctx, const MeshView& m, const std::vector<int32_t>& vfree,
                     int64_t nfree, BlockCSR& A);
// SettleFn: joins every download.
void galerkin_device_settle(void* ctx);
// WaitFn: the products' structures reach the host on threads of their own.
void galerkin_device_wait_structure(void* ctx, int level);
// Takes ownership of level l's prolongation on the device (stream-ordered
// allocations on the context's stream; int64 row pointers, int32 columns, FP64
// weights): the product from level l then uses it (and its transpose, built on
// the device) instead of uploading the host copy.
void galerkin_device_adopt_prolongation(GalerkinDevice* g, int level, int64_t nrows, int64_t ncols,
                                        int64_t nnz, int64_t* ptr, int32_t* col, double* val);
// Transpose of a scalar CSR matrix on the device (tree.hip): the entries of each
// column in row order, as a sequential transpose gives them. Device pointers,
// enqueued on stream.
void transpose_device(void* stream, int64_t nrows, int64_t ncols, int64_t nnz, const int64_t* ptr,
                      const int32_t* col, const double* val, int64_t* tptr, int32_t* tcol, double* tval);
// Vertex -> element lists of a mesh on the device (tree.hip), as the host's
// vertex_elements (elements ascending per vertex): elems [ne][nvpe], vptr
// [nv + 1], velem [ne * nvpe], device pointers; enqueued on stream.
void vertex_elements_device(void* stream, const int32_t* elems, int64_t ne, int nvpe, int64_t nv,
                            int64_t* vptr, int32_t* velem);
// TransfersFn on the device (tree.hip), on the context's stream: false for trees
// deeper than packed 64-bit lattice keys allow (21 levels in 3D, 32 in 2D).
bool transfers_device(void* ctx, const MeshView& m, const std::vector<int32_t>& tree_vtx,
                      const std::vector<int32_t>& free_vertices, const std::vector<int32_t>& pos_in_tree,
                      int capacity, Transfers& out);
// Starts the background downloads of the products' values into the host
// hierarchy (levels other than the coarsest, whose values arrive at once);
// free_after: each level's device copy is released once its values are home.
void galerkin_device_start_downloads(GalerkinDevice* g, bool free_after);
// Starts any download not started yet (keeping the device copies) and waits for
// all of them; throws their error, if any.
void galerkin_device_join(GalerkinDevice* g);

// A level's canonical FP64 operator on the device (block CSR: int64 row
// pointers, int32 columns, row-major d x d blocks).
struct DevOperator {
  int64_t n = 0;
  const int64_t* ptr = nullptr;
  const int32_t* col = nullptr;
  const double* val = nullptr;
};
// Level l's resident operator from the device Galerkin products; false if none.
bool galerkin_device_operator(const GalerkinDevice* g, int l, DevOperator* out);
// The context's stream (a hipStream_t).
void* galerkin_device_stream(const GalerkinDevice* g);
// Level l's canonical prolongation (int64 row pointers, int32 columns, FP64
// weights), kept on the device after the level's Galerkin product for the
// upload, on the context's stream; false when there is none. Released by
// galerkin_device_release_prolongation or with the context.
bool galerkin_device_prolongation(GalerkinDevice* g, int level, int64_t* nrows, int64_t* ncols,
                                  int64_t* nnz, const int64_t** ptr, const int32_t** col,
                                  const double** val);
void galerkin_device_release_prolongation(GalerkinDevice* g, int level);
// A level's transfers in device numbering from its canonical prolongation on
// the device (tree.hip): row i of P is canonical row perm[i], its columns
// renumbered by inv_next in their canonical order; P^T the stable transpose
// (entries of a column in row order); 32-bit row pointers; weights copied
// (pw64, tw64) and rounded to FP32 (pw32, tw32) where those are non-null. The
// arrays the host's upload builds, bit for bit. Device pointers, on stream.
void transfers_layout_device(void* stream, int64_t n, int64_t nn, int64_t nnz, const int64_t* ptr,
                             const int32_t* col, const double* val, const int32_t* perm,
                             const int32_t* inv_next, int32_t* pptr, int32_t* pidx, double* pw64,
                             float* pw32, int32_t* tptr, int32_t* tidx, double* tw64, float* tw32);

// Device layout of one level from its canonical operator A (device pointers;
// the level's device rows i = 0..n-1 map to canonical rows perm[i], canonical
// columns to device columns by inv; [lo[i], hi[i]) is row i's cell and
// [blo[i], bhi[i]) its colour block, the cell when blo / bhi are null).
// Off-cell blocks fall into four parts by device column j:
//   L: j < blo (earlier colours), E: blo <= j < lo (earlier cells of the block),
//   F: hi <= j < bhi (later cells of the block), U: j >= bhi (later colours).
//   count: cnt of each part per row (E / F only where their cnt is non-null);
//   fill:  each part's rows at its ptr (padded entries: column i, zero blocks),
//          columns ascending, values plane-major with stride n in the requested
//          precisions; in-cell blocks into the dense cell matrices (cell_of_row
//          non-null: column-major NU x NU per cell, NU = 2^d d) or the diagonal
//          blocks (cell_of_row null). M32 / M64 are zeroed first. The diagonal
//          entry of a constrained component (fixed non-null) is set to 1 (its
//          row and column are zero in A).
// Both are enqueued on `stream` (a hipStream_t; null = the null stream) and
// return after it has finished them.
enum { kPartL = 0, kPartE = 1, kPartF = 2, kPartU = 3, kParts = 4 };
struct LayoutPart {
  const int* ptr = nullptr;
  int* cnt = nullptr;
  int64_t n = 0;        // stored entries (plane stride)
  int* col = nullptr;
  float* v32 = nullptr;
  double* v64 = nullptr;
};
struct LayoutArgs {
  int d = 0;   // 2 or 3
  int n = 0;
  const int *perm = nullptr, *inv = nullptr, *lo = nullptr, *hi = nullptr;
  const int *blo = nullptr, *bhi = nullptr;
  const int* cell_of_row = nullptr;
  const uint8_t* fixed = nullptr;   // per device row: constrained components (unit diagonal)
  LayoutPart part[kParts];
  float* M32 = nullptr;
  double* M64 = nullptr;
  int64_t m_len = 0;   // elements of M32 / M64
};
void layout_count(const DevOperator& A, const LayoutArgs& a, void* stream);
void layout_fill(const DevOperator& A, const LayoutArgs& a, void* stream);

// Builds the whole hierarchy on the host. Throws vasmg::Error.
void build_hierarchy(const MeshView& mesh, const SetupParams& prm, Hierarchy& out);

// Block-diagonal union of finished hierarchies of the same dimension (no colour
// blocks): level l holds level l of every part, a shallower part padded with
// copies of its coarsest level (identity prolongations, point Gauss-Seidel);
// the coarsest factor is the parts' factors on the diagonal; the union's mesh
// vertices are the parts' one after the other. Throws vasmg::Error.
void pack_hierarchies(const std::vector<const Hierarchy*>& parts, Hierarchy& out);

// Damped vertex-block Jacobi smoother data: inverse diagonal blocks [n][d][d]
// (canonical order) and the largest eigenvalue of D^{-1} A by power iteration.
void block_diag_inverse(const BlockCSR& A, const std::vector<uint8_t>& fixed,
                        std::vector<double>& out);
double jacobi_lambda_max(const BlockCSR& A, const std::vector<double>& dinv, int iters);

}  // namespace vasmg
