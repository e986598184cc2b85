// Host setup of the V-ASMG hierarchy (arXiv 2505.09064, Section 3 setup step).
//
//  * P1 stiffness assembly in d x d blocks over the free vertices (Section 2:
//    weak form a(u,v) = int 2 mu eps(u):eps(v) + lambda div u div v with the
//    Lame constants of Section 2; plane strain in 2D).
//  * Region tree (Section 3.1.1 Steps 1-3): root square/cube from one min and
//    one max over all coordinates; a node holding more than `capacity` vertices
//    splits into 2^d children; a vertex goes to the upper child along an axis
//    iff its coordinate is >= the midline. Node geometry lives on an integer
//    lattice: depth-i nodes (root depth 1) have side 2^(48-i) and key K maps to
//    m + (M - m) * (K * 2^-47), so midlines are reproducible bit for bit.
//  * Level 1 vertices: corners of the non-empty leaves; fine-to-level-1
//    prolongation by bilinear/trilinear interpolation in the leaf
//    (Section 3.1.1 Step 4, Section 3.2, weights read as 1 - |dx|/h per axis).
//  * Coarser levels (Section 3.1.2): the deepest regions merge into their
//    parents until only the root is left; a vertex of the next level is
//    injected, any other vertex is interpolated in its merged parent.
//  * Prolongation columns with no nonzero weight are dropped.
//  * Galerkin operators A_{l+1} = P_l^T A_l P_l (Section 3, equations (R), (Ac))
//    by a row-wise block SpGEMM over the structural pattern.
//  * Gauss-Seidel visiting order (not part of the paper): single-vertex cells
//    on the fine level, lattice cells of twice the finest spacing on coarse
//    levels, greedy first-fit colouring of the cells (fewest colours among the
//    canonical and mod-2 / mod-3 lattice-class visiting orders).
//  * Dense Cholesky factor of the coarsest operator (Section 3 Step 2.3).
//
// Must be compiled without floating-point contraction (-ffp-contract=off):
// tree decisions and level-1 weights are compared bit for bit with an
// independent implementation.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <numeric>
#include <thread>
#include <utility>

#include "hierarchy.hpp"

#ifdef _OPENMP
#include <omp.h>
#include <parallel/algorithm>
#endif

namespace vasmg {
namespace {

constexpr int kMaxDepth = 48;          // depth-48 nodes have side 1 key unit
constexpr double kKeyScale = 0x1p-47;  // keys in [0, 2^47]

[[noreturn]] void fail(int status, const std::string& msg) { throw Error{status, msg}; }

inline uint64_t side_of(int depth) { return uint64_t(1) << (kMaxDepth - depth); }

// canonical vertex order: lexicographic in (z, y, x)
inline bool key_less(const Key& a, const Key& b) {
  if (a[2] != b[2]) return a[2] < b[2];
  if (a[1] != b[1]) return a[1] < b[1];
  return a[0] < b[0];
}

struct Region {
  int depth;
  Key lo;
};
inline bool region_less(const Region& a, const Region& b) {
  if (a.depth != b.depth) return a.depth < b.depth;
  return key_less(a.lo, b.lo);
}
inline bool region_eq(const Region& a, const Region& b) {
  return a.depth == b.depth && a.lo == b.lo;
}

// --------------------------------------------------------------------------
// validation
// --------------------------------------------------------------------------
void validate(const MeshView& m) {
  if (m.d != 2 && m.d != 3) fail(1, "dim must be 2 or 3");
  if (m.nv <= 0 || m.ne <= 0) fail(1, "mesh has no vertices or no elements");
  if (m.nv >= (int64_t(1) << 31) / 3) fail(1, "too many vertices for int32 indexing");
  if (!m.coords || !m.elems || !m.E || !m.nu || !m.fixed) fail(1, "null mesh array");
  const int d = m.d;
  const int64_t nvd = m.nv * d;
  int bad_coord = 0, bad_flag = 0;
#pragma omp parallel for schedule(static) reduction(| : bad_coord, bad_flag)
  for (int64_t i = 0; i < nvd; ++i) {
    bad_coord |= std::isfinite(m.coords[i]) ? 0 : 1;
    bad_flag |= m.fixed[i] > 1 ? 1 : 0;
  }
  if (bad_coord) fail(1, "non-finite vertex coordinate");
  if (bad_flag) fail(1, "fixed flags must be 0 or 1");
  // the first invalid element (found in parallel), then its first failing check
  auto element_ok = [&](int64_t e) {
    if (!(m.E[e] > 0.0) || !std::isfinite(m.E[e])) return false;
    if (!(m.nu[e] > -1.0 && m.nu[e] < 0.5)) return false;
    for (int a = 0; a <= d; ++a) {
      const int32_t v = m.elems[e * (d + 1) + a];
      if (v < 0 || v >= m.nv) return false;
    }
    return true;
  };
  int64_t first = m.ne;
#pragma omp parallel for schedule(static) reduction(min : first)
  for (int64_t e = 0; e < m.ne; ++e)
    if (!element_ok(e)) first = std::min(first, e);
  if (first < m.ne) {
    const int64_t e = first;
    if (!(m.E[e] > 0.0) || !std::isfinite(m.E[e])) fail(1, "E must be finite and > 0");
    if (!(m.nu[e] > -1.0 && m.nu[e] < 0.5)) fail(1, "nu must lie in (-1, 0.5)");
    fail(1, "element vertex index out of range");
  }
}

// --------------------------------------------------------------------------
// P1 element stiffness
// --------------------------------------------------------------------------
// Gradients of the barycentric functions: with X the matrix of edge vectors
// x_a - x_0 (rows), grad lambda_a = row a of X^{-T}; grad lambda_0 = -sum.
// Returns the signed determinant of X.
double p1_grads(int d, const double* xs[4], double G[4][3]) {
  double X[3][3] = {{0}};
  for (int a = 0; a < d; ++a)
    for (int k = 0; k < d; ++k) X[a][k] = xs[a + 1][k] - xs[0][k];
  double det, inv[3][3];
  if (d == 2) {
    det = X[0][0] * X[1][1] - X[0][1] * X[1][0];
    inv[0][0] = X[1][1] / det;  inv[0][1] = -X[0][1] / det;
    inv[1][0] = -X[1][0] / det; inv[1][1] = X[0][0] / det;
  } else {
    const double c00 = X[1][1] * X[2][2] - X[1][2] * X[2][1];
    const double c01 = X[1][2] * X[2][0] - X[1][0] * X[2][2];
    const double c02 = X[1][0] * X[2][1] - X[1][1] * X[2][0];
    det = X[0][0] * c00 + X[0][1] * c01 + X[0][2] * c02;
    inv[0][0] = c00 / det;
    inv[1][0] = c01 / det;
    inv[2][0] = c02 / det;
    inv[0][1] = (X[0][2] * X[2][1] - X[0][1] * X[2][2]) / det;
    inv[1][1] = (X[0][0] * X[2][2] - X[0][2] * X[2][0]) / det;
    inv[2][1] = (X[0][1] * X[2][0] - X[0][0] * X[2][1]) / det;
    inv[0][2] = (X[0][1] * X[1][2] - X[0][2] * X[1][1]) / det;
    inv[1][2] = (X[0][2] * X[1][0] - X[0][0] * X[1][2]) / det;
    inv[2][2] = (X[0][0] * X[1][1] - X[0][1] * X[1][0]) / det;
  }
  // G[a+1][k] = (X^{-T})[a][k] = inv[k][a]
  for (int a = 0; a < d; ++a)
    for (int k = 0; k < d; ++k) G[a + 1][k] = inv[k][a];
  for (int k = 0; k < d; ++k) {
    double s = 0.0;
    for (int a = 1; a <= d; ++a) s += G[a][k];
    G[0][k] = -s;
  }
  return det;
}

// --------------------------------------------------------------------------
// fine-level assembly
// --------------------------------------------------------------------------
}  // namespace

void vertex_elements(const MeshView& m, std::vector<int64_t>& vptr, std::vector<int64_t>& velem) {
  const int nvpe = m.d + 1;
  vptr.assign(m.nv + 1, 0);
  for (int64_t e = 0; e < m.ne; ++e)
    for (int a = 0; a < nvpe; ++a) vptr[m.elems[e * nvpe + a] + 1]++;
  for (int64_t v = 0; v < m.nv; ++v) vptr[v + 1] += vptr[v];
  velem.assign(vptr[m.nv], 0);
  std::vector<int64_t> fill(vptr.begin(), vptr.end() - 1);
  for (int64_t e = 0; e < m.ne; ++e)
    for (int a = 0; a < nvpe; ++a) velem[fill[m.elems[e * nvpe + a]]++] = e;
}

namespace {

void assemble_fine(const MeshView& m, const std::vector<int32_t>& vfree, int64_t nfree,
                   BlockCSR& A) {
  const int d = m.d, nvpe = d + 1, dd = d * d;
  std::vector<int64_t> vptr, velem;
  vertex_elements(m, vptr, velem);
  std::vector<int32_t> fine2mesh(nfree);
  for (int64_t v = 0; v < m.nv; ++v)
    if (vfree[v] >= 0) fine2mesh[vfree[v]] = static_cast<int32_t>(v);

  // structural pattern: free vertices sharing an element (incl. self)
  A.n = nfree;
  A.d = d;
  A.rowptr.assign(nfree + 1, 0);
  std::vector<std::vector<int32_t>> rows(nfree);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < nfree; ++i) {
    const int32_t v = fine2mesh[i];
    auto& r = rows[i];
    for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k) {
      const int64_t e = velem[k];
      for (int a = 0; a < nvpe; ++a) {
        const int32_t f = vfree[m.elems[e * nvpe + a]];
        if (f >= 0) r.push_back(f);
      }
    }
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
  }
  for (int64_t i = 0; i < nfree; ++i) A.rowptr[i + 1] = A.rowptr[i] + rows[i].size();
  A.col.resize(A.rowptr[nfree]);
  for (int64_t i = 0; i < nfree; ++i)
    std::copy(rows[i].begin(), rows[i].end(), A.col.begin() + A.rowptr[i]);
  rows.clear();
  rows.shrink_to_fit();
  A.val.assign(A.col.size() * dd, 0.0);

  // values: each row gathers the element matrices of its elements, so rows
  // are independent and the result does not depend on the thread count
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < nfree; ++i) {
    const int32_t v = fine2mesh[i];
    for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k) {
      const int64_t e = velem[k];
      const int32_t* ev = m.elems + e * nvpe;
      const double* xs[4];
      for (int a = 0; a < nvpe; ++a) xs[a] = m.coords + int64_t(ev[a]) * d;
      double G[4][3];
      const double det = p1_grads(d, xs, G);
      const double vol = std::fabs(det) / (d == 2 ? 2.0 : 6.0);
      const double E = m.E[e], nu = m.nu[e];
      const double mu = E / (2.0 * (1.0 + nu));
      const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
      int la = 0;
      while (ev[la] != v) ++la;
      for (int b = 0; b < nvpe; ++b) {
        const int32_t fj = vfree[ev[b]];
        if (fj < 0) continue;
        const int32_t* c0 = A.col.data() + A.rowptr[i];
        const int32_t* c1 = A.col.data() + A.rowptr[i + 1];
        const int64_t pos = (std::lower_bound(c0, c1, fj) - A.col.data());
        double* blk = A.val.data() + pos * dd;
        double gab = 0.0;
        for (int k = 0; k < d; ++k) gab += G[la][k] * G[b][k];
        for (int ci = 0; ci < d; ++ci)
          for (int cj = 0; cj < d; ++cj) {
            double t = mu * G[la][cj] * G[b][ci] + lam * G[la][ci] * G[b][cj];
            if (ci == cj) t += mu * gab;
            blk[ci * d + cj] += vol * t;
          }
      }
    }
  }
}

// --------------------------------------------------------------------------
// region tree
// --------------------------------------------------------------------------
struct TreeResult {
  double m, M;
  int max_depth;
  std::vector<int32_t> leaf_depth;   // per tree vertex
  std::vector<Key> leaf_lo;
};

void build_tree(const double* coords, const std::vector<int32_t>& tree_vtx, int d, int cap,
                TreeResult& T) {
  const int64_t N = static_cast<int64_t>(tree_vtx.size());
  double m = coords[int64_t(tree_vtx[0]) * d], M = m;
  for (int64_t i = 0; i < N; ++i)
    for (int a = 0; a < d; ++a) {
      const double x = coords[int64_t(tree_vtx[i]) * d + a];
      m = std::min(m, x);
      M = std::max(M, x);
    }
  T.m = m;
  T.M = M;
  T.leaf_depth.assign(N, 0);
  T.leaf_lo.assign(N, Key{0, 0, 0});
  T.max_depth = 1;
  const double S = M - m;
  auto keycoord = [&](uint64_t K) { return m + S * (static_cast<double>(K) * kKeyScale); };

  std::vector<int32_t> idx(N), tmp(N);
  std::iota(idx.begin(), idx.end(), 0);
  struct Node {
    int depth;
    Key lo;
    int64_t b, e;
  };
  std::vector<Node> stack;
  stack.push_back({1, Key{0, 0, 0}, 0, N});
  const int nch = 1 << d;
  while (!stack.empty()) {
    Node nd = stack.back();
    stack.pop_back();
    const int64_t cnt = nd.e - nd.b;
    if (cnt <= cap) {
      for (int64_t i = nd.b; i < nd.e; ++i) {
        T.leaf_depth[idx[i]] = nd.depth;
        T.leaf_lo[idx[i]] = nd.lo;
      }
      T.max_depth = std::max(T.max_depth, nd.depth);
      continue;
    }
    if (nd.depth >= kMaxDepth)
      fail(1, "region tree exceeds its depth limit (duplicate vertices?)");
    const uint64_t half = side_of(nd.depth + 1);
    double mid[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) mid[a] = keycoord(nd.lo[a] + half);
    int64_t count[8] = {0};
    for (int64_t i = nd.b; i < nd.e; ++i) {
      const double* x = coords + int64_t(tree_vtx[idx[i]]) * d;
      int c = 0;
      for (int a = 0; a < d; ++a) c |= (x[a] >= mid[a] ? 1 : 0) << a;
      tmp[i] = c;
      count[c]++;
    }
    int64_t start[9];
    start[0] = nd.b;
    for (int c = 0; c < nch; ++c) start[c + 1] = start[c] + count[c];
    {
      std::vector<int32_t> part(cnt);
      int64_t fillp[8];
      for (int c = 0; c < nch; ++c) fillp[c] = start[c] - nd.b;
      for (int64_t i = nd.b; i < nd.e; ++i) part[fillp[tmp[i]]++] = idx[i];
      std::copy(part.begin(), part.end(), idx.begin() + nd.b);
    }
    for (int c = 0; c < nch; ++c) {
      if (count[c] == 0) continue;
      Node ch{nd.depth + 1, nd.lo, start[c], start[c + 1]};
      for (int a = 0; a < d; ++a)
        if ((c >> a) & 1) ch.lo[a] += half;
      stack.push_back(ch);
    }
  }
}

// --------------------------------------------------------------------------
// prolongation assembly helpers
// --------------------------------------------------------------------------
struct Triplet {
  int64_t row;
  Key key;
  double w;
};

// Builds P from (row, column key, weight) triplets with nonzero weights; the
// columns are the distinct keys in canonical order. Returns the column keys.
std::vector<Key> triplets_to_csr(std::vector<Triplet>& tr, int64_t nrows, ScalarCSR& P) {
  const int64_t nt = static_cast<int64_t>(tr.size());
  std::vector<Key> keys(nt);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < nt; ++t) keys[t] = tr[t].key;
  // equal keys are identical, so the sorted distinct keys do not depend on the
  // thread count
  __gnu_parallel::sort(keys.begin(), keys.end(), key_less);
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  P.nrows = nrows;
  P.ncols = static_cast<int64_t>(keys.size());
  P.rowptr.assign(nrows + 1, 0);
  for (const auto& t : tr) P.rowptr[t.row + 1]++;
  for (int64_t i = 0; i < nrows; ++i) P.rowptr[i + 1] += P.rowptr[i];
  std::vector<int32_t> colof(nt);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < nt; ++t)
    colof[t] = static_cast<int32_t>(std::lower_bound(keys.begin(), keys.end(), tr[t].key, key_less) -
                                    keys.begin());
  P.col.assign(nt, 0);
  P.val.assign(nt, 0.0);
  std::vector<int64_t> fill(P.rowptr.begin(), P.rowptr.end() - 1);
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t p = fill[tr[t].row]++;
    P.col[p] = colof[t];
    P.val[p] = tr[t].w;
  }
  // columns ascending within each row (distinct within a row)
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t i = 0; i < nrows; ++i) {
    const int64_t b = P.rowptr[i], e = P.rowptr[i + 1];
    std::pair<int32_t, double> r[64];
    const int64_t len = e - b;
    if (len > 64) {
      std::vector<std::pair<int32_t, double>> v;
      for (int64_t p = b; p < e; ++p) v.emplace_back(P.col[p], P.val[p]);
      std::sort(v.begin(), v.end());
      for (int64_t p = b; p < e; ++p) {
        P.col[p] = v[p - b].first;
        P.val[p] = v[p - b].second;
      }
      continue;
    }
    for (int64_t p = b; p < e; ++p) r[p - b] = {P.col[p], P.val[p]};
    std::sort(r, r + len);
    for (int64_t p = b; p < e; ++p) {
      P.col[p] = r[p - b].first;
      P.val[p] = r[p - b].second;
    }
  }
  return keys;
}

std::vector<Key> region_corners(const std::vector<Region>& R, int d) {
  std::vector<Key> out;
  out.reserve(R.size() << d);
  for (const auto& r : R) {
    const uint64_t s = side_of(r.depth);
    for (int b = 0; b < (1 << d); ++b) {
      Key k = r.lo;
      for (int a = 0; a < d; ++a)
        if ((b >> a) & 1) k[a] += s;
      out.push_back(k);
    }
  }
  __gnu_parallel::sort(out.begin(), out.end(), key_less);
  out.erase(std::unique(out.begin(), out.end()), out.end());
  return out;
}

// --------------------------------------------------------------------------
// Galerkin product A_c = P^T A P (block, weights shared by the components)
// --------------------------------------------------------------------------
void galerkin(const BlockCSR& A, const ScalarCSR& P, BlockCSR& Ac) {
  const int d = A.d, dd = d * d;
  const int64_t nc = P.ncols;
  // P^T (rows = coarse vertices)
  ScalarCSR PT;
  PT.nrows = nc;
  PT.ncols = P.nrows;
  PT.rowptr.assign(nc + 1, 0);
  for (int32_t c : P.col) PT.rowptr[c + 1]++;
  for (int64_t i = 0; i < nc; ++i) PT.rowptr[i + 1] += PT.rowptr[i];
  PT.col.resize(P.col.size());
  PT.val.resize(P.col.size());
  {
    std::vector<int64_t> fill(PT.rowptr.begin(), PT.rowptr.end() - 1);
    for (int64_t r = 0; r < P.nrows; ++r)
      for (int64_t p = P.rowptr[r]; p < P.rowptr[r + 1]; ++p) {
        const int64_t q = fill[P.col[p]]++;
        PT.col[q] = static_cast<int32_t>(r);
        PT.val[q] = P.val[p];
      }
  }
  std::vector<std::vector<int32_t>> rcol(nc);
  std::vector<std::vector<double>> rval(nc);
#pragma omp parallel
  {
    std::vector<int64_t> pos(nc, -1);
    std::vector<int32_t> cols;
    std::vector<double> acc;
#pragma omp for schedule(dynamic, 256)
    for (int64_t I = 0; I < nc; ++I) {
      cols.clear();
      acc.clear();
      for (int64_t p = PT.rowptr[I]; p < PT.rowptr[I + 1]; ++p) {
        const int32_t k = PT.col[p];
        const double wk = PT.val[p];
        for (int64_t q = A.rowptr[k]; q < A.rowptr[k + 1]; ++q) {
          const int32_t l = A.col[q];
          const double* blk = A.val.data() + q * dd;
          for (int64_t s = P.rowptr[l]; s < P.rowptr[l + 1]; ++s) {
            const int32_t J = P.col[s];
            const double w = wk * P.val[s];
            int64_t at = pos[J];
            if (at < 0) {
              at = static_cast<int64_t>(cols.size());
              pos[J] = at;
              cols.push_back(J);
              acc.resize(acc.size() + dd, 0.0);
            }
            double* dst = acc.data() + at * dd;
            for (int t = 0; t < dd; ++t) dst[t] += w * blk[t];
          }
        }
      }
      std::vector<int64_t> order(cols.size());
      std::iota(order.begin(), order.end(), 0);
      std::sort(order.begin(), order.end(),
                [&](int64_t a, int64_t b) { return cols[a] < cols[b]; });
      auto& oc = rcol[I];
      auto& ov = rval[I];
      oc.resize(cols.size());
      ov.resize(cols.size() * dd);
      for (size_t t = 0; t < order.size(); ++t) {
        oc[t] = cols[order[t]];
        std::memcpy(ov.data() + t * dd, acc.data() + order[t] * dd, sizeof(double) * dd);
      }
      for (int32_t J : cols) pos[J] = -1;
    }
  }
  Ac.n = nc;
  Ac.d = d;
  Ac.rowptr.assign(nc + 1, 0);
  for (int64_t I = 0; I < nc; ++I) Ac.rowptr[I + 1] = Ac.rowptr[I] + rcol[I].size();
  Ac.col.resize(Ac.rowptr[nc]);
  Ac.val.resize(Ac.rowptr[nc] * dd);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t I = 0; I < nc; ++I) {
    std::copy(rcol[I].begin(), rcol[I].end(), Ac.col.begin() + Ac.rowptr[I]);
    std::copy(rval[I].begin(), rval[I].end(), Ac.val.begin() + Ac.rowptr[I] * dd);
  }
}

// --------------------------------------------------------------------------
// Gauss-Seidel order: cells and their greedy first-fit colouring
// --------------------------------------------------------------------------
// First fit over the graph (ptr, adj) visiting the nodes in `order`; self
// loops are ignored (a node is uncoloured when visited).
int32_t greedy_color_in_order(const std::vector<int64_t>& ptr, const int32_t* adj,
                              const std::vector<int64_t>& order, std::vector<int32_t>& color) {
  const int64_t n = static_cast<int64_t>(ptr.size()) - 1;
  color.assign(n, -1);
  std::vector<int64_t> stamp;
  int32_t ncol = 0;
  for (int64_t t = 0; t < n; ++t) {
    const int64_t i = order[t];
    for (int64_t p = ptr[i]; p < ptr[i + 1]; ++p) {
      const int32_t c = color[adj[p]];
      if (c >= 0) {
        if (static_cast<size_t>(c) >= stamp.size()) stamp.resize(c + 1, -1);
        stamp[c] = t;
      }
    }
    int32_t c = 0;
    while (static_cast<size_t>(c) < stamp.size() && stamp[c] == t) ++c;
    color[i] = c;
    ncol = std::max(ncol, c + 1);
  }
  return ncol;
}

// Lattice blocks of side `side` (key units): vertex -> block in canonical order
// of the block keys; returns the sorted block keys.
std::vector<Key> lattice_blocks(const Level& lv, uint64_t side, std::vector<int32_t>& of) {
  const int64_t n = lv.n;
  std::vector<Key> ck(n);
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) ck[i][a] = lv.keys[i][a] / side;
  std::vector<Key> keys = ck;
  __gnu_parallel::sort(keys.begin(), keys.end(), key_less);
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  of.resize(n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    of[i] = static_cast<int32_t>(std::lower_bound(keys.begin(), keys.end(), ck[i], key_less) -
                                 keys.begin());
  return keys;
}

// Fine level: every vertex is a cell and a colour block, coloured in canonical
// order. Coarse lattice levels: cells of side 2 * h (h = the finest region side
// of the level), in canonical order of their cell keys; in 3D with colour
// blocks on, where the couplings reach 3 or 4 steps of h, the cells are grouped
// into blocks of side 4 h (blocks two apart along an axis are then at least 5
// steps apart, so only neighbouring blocks couple and 2^d colours suffice),
// else every cell is its own block. Blocks are coloured greedily; the colouring
// with the fewest colours among the canonical, (block key mod 2)-class and
// (block key mod 3)-class visiting orders is kept (ties keep the earlier order).
void build_gs_order(Level& lv, bool lattice, int d, bool color_blocks) {
  const int64_t n = lv.n;
  std::vector<Key> bkeys;
  if (!lattice) {
    lv.cell.resize(n);
    std::iota(lv.cell.begin(), lv.cell.end(), 0);
    lv.ncells = n;
    lv.block = lv.cell;
    lv.nblocks = n;
    lv.block_steps = 1;
  } else {
    const uint64_t h = side_of(lv.max_region_depth);
    bkeys = lattice_blocks(lv, 2 * h, lv.cell);
    lv.ncells = static_cast<int64_t>(bkeys.size());
    lv.block_steps = 2;
    if (color_blocks && d == 3) {
      uint64_t reach = 0;
#pragma omp parallel for schedule(static) reduction(max : reach)
      for (int64_t i = 0; i < n; ++i)
        for (int64_t p = lv.A.rowptr[i]; p < lv.A.rowptr[i + 1]; ++p) {
          const Key& a = lv.keys[i];
          const Key& b = lv.keys[lv.A.col[p]];
          for (int q = 0; q < 3; ++q) reach = std::max(reach, a[q] > b[q] ? a[q] - b[q] : b[q] - a[q]);
        }
      if (reach > 2 * h && reach <= 4 * h) lv.block_steps = 4;
    }
    if (lv.block_steps == 4) {
      bkeys = lattice_blocks(lv, 4 * h, lv.block);
    } else {
      lv.block = lv.cell;
    }
    lv.nblocks = static_cast<int64_t>(bkeys.size());
  }
  // block adjacency from the structural block pattern (on the fine level, where
  // every vertex is its own block, the pattern itself)
  const int64_t nc = lv.nblocks;
  std::vector<int64_t> gptr;
  std::vector<int32_t> gadj;
  const std::vector<int64_t>* adj_ptr = &gptr;
  if (!lattice) {
    adj_ptr = &lv.A.rowptr;
  } else {
    std::vector<int64_t> vptr(nc + 1, 0);
    for (int64_t i = 0; i < n; ++i) vptr[lv.block[i] + 1]++;
    for (int64_t c = 0; c < nc; ++c) vptr[c + 1] += vptr[c];
    std::vector<int32_t> members(n);
    {
      std::vector<int64_t> fill(vptr.begin(), vptr.end() - 1);
      for (int64_t i = 0; i < n; ++i) members[fill[lv.block[i]]++] = static_cast<int32_t>(i);
    }
    // each block's neighbour list is independent: the distinct neighbour blocks
    // found with a per-thread marker (no sort of the raw entries), then sorted
    gptr.assign(nc + 1, 0);
    std::vector<std::vector<int32_t>> nb(nc);
#pragma omp parallel
    {
      std::vector<int64_t> mark(nc, -1);
#pragma omp for schedule(dynamic, 256)
      for (int64_t c = 0; c < nc; ++c) {
        auto& tmp = nb[c];
        for (int64_t q = vptr[c]; q < vptr[c + 1]; ++q) {
          const int32_t v = members[q];
          for (int64_t p = lv.A.rowptr[v]; p < lv.A.rowptr[v + 1]; ++p) {
            const int32_t b = lv.block[lv.A.col[p]];
            if (mark[b] != c) {
              mark[b] = c;
              tmp.push_back(b);
            }
          }
        }
        std::sort(tmp.begin(), tmp.end());
      }
    }
    for (int64_t c = 0; c < nc; ++c) gptr[c + 1] = gptr[c] + static_cast<int64_t>(nb[c].size());
    gadj.resize(gptr[nc]);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t c = 0; c < nc; ++c) std::copy(nb[c].begin(), nb[c].end(), gadj.begin() + gptr[c]);
  }
  // the candidate visiting orders are coloured side by side; the first order
  // with the fewest colours wins, as in a sequential scan
  const int n_orders = lattice ? 3 : 1;
  std::vector<std::vector<int32_t>> cand(n_orders);
  std::vector<int32_t> ncol(n_orders, 0);
#pragma omp parallel for schedule(static, 1)
  for (int o = 0; o < n_orders; ++o) {
    std::vector<int64_t> order(nc);
    std::iota(order.begin(), order.end(), 0);
    if (o > 0) {
      const int q = o + 1;
      std::vector<int64_t> cls(nc, 0);
      for (int64_t c = 0; c < nc; ++c) {
        int64_t w = 1;
        for (int a = 0; a < d; ++a) {
          cls[c] += static_cast<int64_t>(bkeys[c][a] % q) * w;
          w *= q;
        }
      }
      std::stable_sort(order.begin(), order.end(),
                       [&](int64_t a, int64_t b) { return cls[a] < cls[b]; });
    }
    ncol[o] = greedy_color_in_order(*adj_ptr, lattice ? gadj.data() : lv.A.col.data(), order, cand[o]);
  }
  int best_o = 0;
  for (int o = 1; o < n_orders; ++o)
    if (ncol[o] < ncol[best_o]) best_o = o;
  const int32_t best = ncol[best_o];
  lv.block_color.swap(cand[best_o]);
  lv.ncolors = best;
  lv.color.resize(n);
  for (int64_t i = 0; i < n; ++i) lv.color[i] = lv.block_color[lv.block[i]];
}

// Sets the rows and columns of the constrained components of A to zero.
void zero_constrained(BlockCSR& A, const std::vector<uint8_t>& fixed) {
  if (fixed.empty()) return;
  const int d = A.d, dd = d * d;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) {
      const uint8_t fr = fixed[i], fc = fixed[A.col[p]];
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b)
          if (((fr >> a) & 1) || ((fc >> b) & 1)) A.val[p * dd + a * d + b] = 0.0;
    }
}

// --------------------------------------------------------------------------
// dense Cholesky (lower), FP64
// --------------------------------------------------------------------------
// Lower Cholesky factor of the coarsest operator, with an identity row and
// column at its constrained components.
void dense_cholesky(const BlockCSR& A, const std::vector<uint8_t>& fixed, std::vector<double>& L,
                    int64_t& n) {
  const int d = A.d, dd = d * d;
  n = A.n * d;
  if (n > 20000) fail(1, "coarsest level too large for a dense factorisation");
  std::vector<double> M(n * n, 0.0);
  double maxdiag = 0.0;
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) {
      const int64_t j = A.col[p];
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) M[(i * d + a) * n + j * d + b] = A.val[p * dd + a * d + b];
    }
  if (!fixed.empty())
    for (int64_t i = 0; i < A.n; ++i)
      for (int a = 0; a < d; ++a)
        if ((fixed[i] >> a) & 1) M[(i * d + a) * n + i * d + a] = 1.0;
  for (int64_t i = 0; i < n; ++i) maxdiag = std::max(maxdiag, M[i * n + i]);
  for (int64_t j = 0; j < n; ++j) {
    double s = M[j * n + j];
    for (int64_t k = 0; k < j; ++k) s -= M[j * n + k] * M[j * n + k];
    if (!(s > 1e-12 * maxdiag) || !std::isfinite(s))
      fail(6, "coarsest operator is not positive definite: no DOFs fixed (rigid-body modes), or "
                "fewer free DOFs than the coarser levels' vertices can take (e.g. a mesh with a "
                "single free vertex)");
    const double ljj = std::sqrt(s);
    M[j * n + j] = ljj;
    for (int64_t i = j + 1; i < n; ++i) {
      double t = M[i * n + j];
      for (int64_t k = 0; k < j; ++k) t -= M[i * n + k] * M[j * n + k];
      M[i * n + j] = t / ljj;
    }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j) M[i * n + j] = 0.0;
  L.swap(M);
}

// Point Gauss-Seidel order of a level used as a smoothing level although its
// own hierarchy ends there (a packed part shallower than the others): single
// vertices (a single cell when it has at most 2^d vertices and lies below the
// fine level), greedy first-fit colours in canonical order.
void padded_gs_order(const Level& src, int d, bool fine, Level& out_part) {
  const int64_t n = src.n;
  out_part.cell.resize(n);
  out_part.block.resize(n);
  if (!fine && n <= (int64_t(1) << d)) {
    std::fill(out_part.cell.begin(), out_part.cell.end(), 0);
    out_part.ncells = 1;
    out_part.block_color.assign(1, 0);
    out_part.color.assign(n, 0);
    out_part.ncolors = 1;
  } else {
    std::iota(out_part.cell.begin(), out_part.cell.end(), 0);
    out_part.ncells = n;
    std::vector<int64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::vector<int64_t> ptr(src.A.rowptr.begin(), src.A.rowptr.end());
    out_part.ncolors = greedy_color_in_order(ptr, src.A.col.data(), order, out_part.block_color);
    out_part.color = out_part.block_color;
  }
  out_part.block = out_part.cell;
  out_part.nblocks = out_part.ncells;
}

}  // namespace

// --------------------------------------------------------------------------
// Packing: the block-diagonal union of several hierarchies (independent
// problems solved together). Level l of the union holds level l of every part;
// a part with fewer levels contributes copies of its coarsest level below its
// own depth, joined by identity prolongations and swept as a smoothing level:
// the coarse solve under it is exact, so its V-cycle still returns the coarse
// solution (to rounding). Cells, colour blocks and vertices keep their order
// inside each part (a part's cells before the next part's within a colour);
// the union's "mesh" is the parts' meshes one after the other.
// --------------------------------------------------------------------------
void pack_hierarchies(const std::vector<const Hierarchy*>& parts, Hierarchy& U) {
  if (parts.empty()) fail(1, "nothing to pack");
  const int d = parts[0]->d;
  int Lmax = 0;
  for (const Hierarchy* p : parts) {
    if (p->d != d) fail(1, "packed problems must have the same dimension");
    for (const Level& lv : p->levels)
      if (lv.block_steps > 2) fail(1, "packed problems must not use colour blocks");
    Lmax = std::max(Lmax, static_cast<int>(p->levels.size()) - 1);
  }
  const int np = static_cast<int>(parts.size());
  U = Hierarchy();
  U.d = d;
  U.capacity = parts[0]->capacity;
  int64_t vo = 0;
  for (const Hierarchy* p : parts) {
    for (int32_t v : p->free_vertices) U.free_vertices.push_back(static_cast<int32_t>(v + vo));
    vo += p->n_mesh_vertices;
    U.max_depth = std::max(U.max_depth, p->max_depth);
  }
  if (vo > INT32_MAX) fail(1, "packed problems exceed 2^31 vertices");
  U.n_mesh_vertices = vo;
  auto src_of = [&](int i, int l) {
    return std::min(l, static_cast<int>(parts[i]->levels.size()) - 1);
  };
  U.levels.resize(Lmax + 1);
  for (int l = 0; l <= Lmax; ++l) {
    Level& u = U.levels[l];
    u.A.d = d;
    u.A.rowptr.assign(1, 0);
    bool any_fixed = false;
    for (int i = 0; i < np; ++i) any_fixed = any_fixed || !parts[i]->levels[src_of(i, l)].fixed.empty();
    int64_t off = 0, cell_off = 0;
    const bool coarsest = l == Lmax;
    for (int i = 0; i < np; ++i) {
      const int si = src_of(i, l);
      const Level& s = parts[i]->levels[si];
      const bool padded = si < l || (si == static_cast<int>(parts[i]->levels.size()) - 1 && !coarsest);
      // operator: block diagonal
      const int64_t base = u.A.col.size();
      for (int64_t r = 0; r < s.n; ++r) u.A.rowptr.push_back(base + s.A.rowptr[r + 1]);
      for (int32_t c : s.A.col) u.A.col.push_back(static_cast<int32_t>(c + off));
      u.A.val.insert(u.A.val.end(), s.A.val.begin(), s.A.val.end());
      if (any_fixed) {
        if (s.fixed.empty())
          u.fixed.insert(u.fixed.end(), s.n, 0);
        else
          u.fixed.insert(u.fixed.end(), s.fixed.begin(), s.fixed.end());
      }
      if (!coarsest) {
        // prolongation to the next level: the part's own, or the identity
        const int sn = src_of(i, l + 1);
        int64_t noff = 0;
        for (int j = 0; j < i; ++j) noff += parts[j]->levels[src_of(j, l + 1)].n;
        ScalarCSR& P = u.P;
        if (P.rowptr.empty()) P.rowptr.assign(1, 0);
        if (sn > si) {
          const int64_t pb = P.col.size();
          for (int64_t r = 0; r < s.n; ++r) P.rowptr.push_back(pb + s.P.rowptr[r + 1]);
          for (int32_t c : s.P.col) P.col.push_back(static_cast<int32_t>(c + noff));
          P.val.insert(P.val.end(), s.P.val.begin(), s.P.val.end());
        } else {
          for (int64_t r = 0; r < s.n; ++r) {
            P.col.push_back(static_cast<int32_t>(r + noff));
            P.val.push_back(1.0);
            P.rowptr.push_back(static_cast<int64_t>(P.col.size()));
          }
        }
        // Gauss-Seidel order: the part's own, or point order on a padded level
        Level pad;
        const Level* g = &s;
        if (padded) {
          padded_gs_order(s, d, l == 0, pad);
          g = &pad;
        }
        for (int64_t r = 0; r < s.n; ++r) {
          u.cell.push_back(static_cast<int32_t>(g->cell[r] + cell_off));
          u.color.push_back(g->color[r]);
        }
        for (int64_t c = 0; c < g->ncells; ++c) u.block_color.push_back(g->block_color[c]);
        cell_off += g->ncells;
        u.ncolors = std::max(u.ncolors, g->ncolors);
      }
      off += s.n;
    }
    u.n = off;
    u.A.n = off;
    if (!coarsest) {
      u.P.nrows = off;
      int64_t nn = 0;
      for (int i = 0; i < np; ++i) nn += parts[i]->levels[src_of(i, l + 1)].n;
      u.P.ncols = nn;
      u.ncells = cell_off;
      u.block = u.cell;
      u.nblocks = cell_off;
      u.block_steps = l == 0 ? 1 : 2;
    } else {
      u.color.assign(off, 0);
      u.ncolors = 0;
    }
  }
  // coarsest factor: the parts' own factors on the diagonal
  int64_t nc = 0;
  for (const Hierarchy* p : parts) nc += p->n_coarse_dofs;
  if (nc > 4096) fail(1, "packed coarsest levels exceed 4096 DOFs");
  U.n_coarse_dofs = nc;
  U.chol.assign(static_cast<size_t>(nc * nc), 0.0);
  int64_t o = 0;
  for (const Hierarchy* p : parts) {
    const int64_t m = p->n_coarse_dofs;
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j <= i; ++j) U.chol[(o + i) * nc + o + j] = p->chol[i * m + j];
    o += m;
  }
}

// --------------------------------------------------------------------------
void build_hierarchy(const MeshView& m, const SetupParams& prm, Hierarchy& H) {
  validate(m);
  if (prm.capacity < 1) fail(1, "leaf_capacity must be >= 1");
  const int d = m.d;
  H = Hierarchy();
  H.d = d;
  H.n_mesh_vertices = m.nv;
  H.capacity = prm.capacity;
  auto t0 = std::chrono::steady_clock::now();
  auto mark = [&](const char* phase) {
    const auto t1 = std::chrono::steady_clock::now();
    H.phase_ms.emplace_back(phase, std::chrono::duration<double, std::milli>(t1 - t0).count());
    t0 = t1;
  };

  // free vertices: those with at least one unconstrained component (fine
  // canonical order = ascending mesh index); fully fixed vertices are eliminated
  std::vector<int32_t> vfree(m.nv, -1);
  int64_t nfree = 0;
  std::vector<uint8_t> fixed0;
  bool partial = false;
  for (int64_t v = 0; v < m.nv; ++v) {
    uint8_t bits = 0;
    for (int a = 0; a < d; ++a)
      if (m.fixed[v * d + a]) bits |= static_cast<uint8_t>(1u << a);
    if (bits == (1u << d) - 1) continue;
    vfree[v] = static_cast<int32_t>(nfree++);
    H.free_vertices.push_back(static_cast<int32_t>(v));
    fixed0.push_back(bits);
    partial = partial || bits != 0;
  }
  if (nfree == 0) fail(1, "every vertex is fixed: nothing to solve");
  int64_t bad = m.ne;   // first inverted or degenerate element, if any
#pragma omp parallel for schedule(static) reduction(min : bad)
  for (int64_t e = 0; e < m.ne; ++e) {
    const double* xs[4];
    for (int a = 0; a <= d; ++a) xs[a] = m.coords + int64_t(m.elems[e * (d + 1) + a]) * d;
    double G[4][3];
    const double det = p1_grads(d, xs, G);
    if (!(det > 0.0) || !std::isfinite(det)) bad = std::min(bad, e);
  }
  if (bad < m.ne) fail(1, "element " + std::to_string(bad) + " is inverted or degenerate");

  // Levels never move once created (callbacks keep pointers to their operators):
  // one level per tree depth at most, plus the fine level.
  H.levels.reserve(kMaxDepth + 2);
  H.levels.emplace_back();
  {
    Level& L0 = H.levels.back();
    L0.n = nfree;
    if (partial) L0.fixed = fixed0;
    if (prm.assemble) {
      prm.assemble(prm.galerkin_ctx, m, vfree, nfree, L0.A);   // constrained rows zeroed there
    } else {
      assemble_fine(m, vfree, nfree, L0.A);
      zero_constrained(L0.A, L0.fixed);
    }
  }
  mark("validate+assemble");

  // ---- region tree over the tree vertices (Section 3.1.1 Steps 1-2)
  std::vector<int32_t> tree_vtx;
  for (int64_t v = 0; v < m.nv; ++v)
    if (!prm.tree_free_only || vfree[v] >= 0) tree_vtx.push_back(static_cast<int32_t>(v));
  std::vector<int32_t> pos_in_tree(m.nv, -1);
  for (size_t i = 0; i < tree_vtx.size(); ++i) pos_in_tree[tree_vtx[i]] = static_cast<int32_t>(i);
  Transfers X;
  if (prm.transfers &&
      prm.transfers(prm.galerkin_ctx, m, tree_vtx, H.free_vertices, pos_in_tree, prm.capacity, X)) {
    H.box_m = X.m;
    H.box_M = X.M;
    H.max_depth = X.max_depth;
    H.levels[0].P = std::move(X.P[0]);
    for (size_t l = 1; l < X.keys.size(); ++l) {
      if (H.levels.size() == H.levels.capacity()) fail(1, "internal error: too many levels");
      H.levels.emplace_back();
      Level& lv = H.levels.back();
      lv.keys = std::move(X.keys[l]);
      lv.n = static_cast<int64_t>(lv.keys.size());
      lv.max_region_depth = X.max_region_depth[l];
      if (l < X.P.size()) lv.P = std::move(X.P[l]);
    }
    mark("tree+P (device)");
  } else {
    TreeResult T;
    build_tree(m.coords, tree_vtx, d, prm.capacity, T);
    mark("tree");
    H.box_m = T.m;
    H.box_M = T.M;
    H.max_depth = T.max_depth;
    const double S = T.M - T.m;
    auto keycoord = [&](uint64_t K) { return T.m + S * (static_cast<double>(K) * kKeyScale); };

    // ---- Step 3: non-empty leaves = level-1 regions
    std::vector<Region> R;
    R.reserve(tree_vtx.size());
    for (size_t i = 0; i < tree_vtx.size(); ++i) R.push_back({T.leaf_depth[i], T.leaf_lo[i]});
    __gnu_parallel::sort(R.begin(), R.end(), region_less);
    R.erase(std::unique(R.begin(), R.end(), region_eq), R.end());

    // ---- Step 4 + Section 3.2: P_0 by multilinear interpolation in the leaf
    std::vector<Key> cur_keys;
    {
      // 2^d slots per row, filled in parallel; zero weights are dropped after
      std::vector<Triplet> tr(static_cast<size_t>(nfree) << d, Triplet{0, Key{0, 0, 0}, 0.0});
  #pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < nfree; ++i) {
        const int32_t v = H.free_vertices[i];
        const int32_t t = pos_in_tree[v];
        const int dep = T.leaf_depth[t];
        const Key lo = T.leaf_lo[t];
        const uint64_t s = side_of(dep);
        double tup[3], tdn[3];
        for (int a = 0; a < d; ++a) {
          const double lc = keycoord(lo[a]);
          const double hc = keycoord(lo[a] + s);
          const double x = m.coords[int64_t(v) * d + a];
          tup[a] = (x - lc) / (hc - lc);
          tdn[a] = (hc - x) / (hc - lc);
        }
        for (int b = 0; b < (1 << d); ++b) {
          double w = 1.0;
          Key k = lo;
          for (int a = 0; a < d; ++a) {
            const bool up = (b >> a) & 1;
            w = w * (up ? tup[a] : tdn[a]);
            if (up) k[a] += s;
          }
          tr[(i << d) + b] = {i, k, w};
        }
      }
      tr.erase(std::remove_if(tr.begin(), tr.end(), [](const Triplet& t) { return t.w == 0.0; }),
               tr.end());
      cur_keys = triplets_to_csr(tr, nfree, H.levels[0].P);
    }
    mark("P0");

    // ---- Section 3.1.2: merge the deepest regions until only the root is left
    while (true) {
      if (H.levels.size() == H.levels.capacity()) fail(1, "internal error: too many levels");
      H.levels.emplace_back();
      Level& lv = H.levels.back();
      lv.n = static_cast<int64_t>(cur_keys.size());
      lv.keys = cur_keys;
      int Dstar = 0;
      for (const auto& r : R) Dstar = std::max(Dstar, r.depth);
      lv.max_region_depth = Dstar;
      if (R.size() == 1 && R[0].depth == 1) break;
      const uint64_t ps = side_of(Dstar - 1);
      std::vector<Region> Rn;
      std::vector<std::pair<Key, Key>> corner_parent;   // corner of a merged region -> parent lo
      for (const auto& r : R) {
        if (r.depth != Dstar) {
          Rn.push_back(r);
          continue;
        }
        Region p{Dstar - 1, r.lo};
        for (int a = 0; a < d; ++a) p.lo[a] = (r.lo[a] / ps) * ps;
        Rn.push_back(p);
        const uint64_t s = side_of(Dstar);
        for (int b = 0; b < (1 << d); ++b) {
          Key k = r.lo;
          for (int a = 0; a < d; ++a)
            if ((b >> a) & 1) k[a] += s;
          corner_parent.emplace_back(k, p.lo);
        }
      }
      __gnu_parallel::sort(Rn.begin(), Rn.end(), region_less);
      Rn.erase(std::unique(Rn.begin(), Rn.end(), region_eq), Rn.end());
      // a total order (corner, then parent): deterministic for any thread count; a
      // corner shared by two merged parents lies on their common face, where both
      // give the same interpolation corners and weights
      __gnu_parallel::sort(corner_parent.begin(), corner_parent.end(),
                           [](const std::pair<Key, Key>& a, const std::pair<Key, Key>& b) {
                             if (a.first != b.first) return key_less(a.first, b.first);
                             return key_less(a.second, b.second);
                           });
      const std::vector<Key> next_all = region_corners(Rn, d);
      // 2^d slots per row, filled in parallel; zero weights are dropped after
      const int64_t ncur = static_cast<int64_t>(cur_keys.size());
      std::vector<Triplet> tr(static_cast<size_t>(ncur) << d, Triplet{0, Key{0, 0, 0}, 0.0});
      int not_corner = 0;
  #pragma omp parallel for schedule(static) reduction(|| : not_corner)
      for (int64_t i = 0; i < ncur; ++i) {
        const Key& kv = cur_keys[i];
        if (std::binary_search(next_all.begin(), next_all.end(), kv, key_less)) {
          tr[i << d] = {i, kv, 1.0};
          continue;
        }
        auto it = std::lower_bound(corner_parent.begin(), corner_parent.end(), kv,
                                   [](const std::pair<Key, Key>& a, const Key& k) {
                                     return key_less(a.first, k);
                                   });
        if (it == corner_parent.end() || it->first != kv) {
          not_corner = 1;
          continue;
        }
        const Key plo = it->second;
        double up[3];
        for (int a = 0; a < d; ++a) {
          const uint64_t rel = kv[a] - plo[a];
          up[a] = rel == ps ? 1.0 : (rel == 0 ? 0.0 : 0.5);
        }
        for (int b = 0; b < (1 << d); ++b) {
          double w = 1.0;
          Key k = plo;
          for (int a = 0; a < d; ++a) {
            const bool hi = (b >> a) & 1;
            w = w * (hi ? up[a] : 1.0 - up[a]);
            if (hi) k[a] += ps;
          }
          tr[(i << d) + b] = {i, k, w};
        }
      }
      if (not_corner) fail(1, "internal error: interpolated vertex is not a corner of a merged region");
      tr.erase(std::remove_if(tr.begin(), tr.end(), [](const Triplet& t) { return t.w == 0.0; }),
               tr.end());
      cur_keys = triplets_to_csr(tr, static_cast<int64_t>(cur_keys.size()), lv.P);
      R.swap(Rn);
    }
    mark("coarse regions+P");
  }

  // constrained components of the coarse levels: a coarse component is
  // constrained when every fine vertex interpolating from it has it fixed
  // (its column of P with the fixed rows zeroed is empty)
  for (size_t l = 0; l + 1 < H.levels.size(); ++l) {
    const Level& f = H.levels[l];
    if (f.fixed.empty()) break;
    Level& c = H.levels[l + 1];
    std::vector<uint8_t> cm(c.n, static_cast<uint8_t>((1u << d) - 1));
    for (int64_t i = 0; i < f.n; ++i)
      for (int64_t p = f.P.rowptr[i]; p < f.P.rowptr[i + 1]; ++p) cm[f.P.col[p]] &= f.fixed[i];
    bool any = false;
    for (uint8_t b : cm) any = any || b != 0;
    if (any) c.fixed.swap(cm);
  }
  if (!H.levels[0].fixed.empty()) mark("coarse constraints");
  // ---- Galerkin operators, with optional truncation of the hierarchy. With the
  // products on the device, each level's Gauss-Seidel order (which needs only its
  // own structure) is built on a host thread of its own while the product from
  // that level runs.
  size_t nlev = H.levels.size();
  std::vector<std::thread> order_threads;
  struct JoinAll {   // joined on every exit, exceptions from the products included
    std::vector<std::thread>& t;
    ~JoinAll() {
      for (auto& x : t)
        if (x.joinable()) x.join();
    }
  } join_guard{order_threads};
  std::vector<std::exception_ptr> order_err(nlev);
  const int nth = omp_get_max_threads();
  for (size_t l = 0; l + 1 < nlev; ++l) {
    if (prm.coarsest_max_dofs > 0 && H.levels[l].n * d <= prm.coarsest_max_dofs) {
      nlev = l + 1;
      break;
    }
    if (prm.galerkin) {
      order_threads.emplace_back([&, l] {
        try {
          omp_set_num_threads(nth);
          if (l > 0 && prm.wait_structure) prm.wait_structure(prm.galerkin_ctx, static_cast<int>(l));
          build_gs_order(H.levels[l], l > 0, d, prm.color_blocks);
        } catch (...) {
          order_err[l] = std::current_exception();
        }
      });
      const bool coarsest =
          l + 2 == nlev || (prm.coarsest_max_dofs > 0 && H.levels[l + 1].n * d <= prm.coarsest_max_dofs);
      prm.galerkin(prm.galerkin_ctx, H.levels[l].A, H.levels[l].P, H.levels[l + 1].A, coarsest);
    } else
      galerkin(H.levels[l].A, H.levels[l].P, H.levels[l + 1].A);
  }
  if (prm.galerkin && prm.wait_structure) prm.wait_structure(prm.galerkin_ctx, -1);
  if (!order_threads.empty()) mark("galerkin (+ordering)");
  for (auto& t : order_threads) t.join();
  for (const auto& e : order_err)
    if (e) std::rethrow_exception(e);
  if (order_threads.empty()) mark("galerkin");
  H.levels.resize(nlev);
  Level& coarsest = H.levels.back();
  coarsest.P = ScalarCSR();
  coarsest.color.assign(coarsest.n, 0);
  coarsest.ncolors = 0;
  if (order_threads.empty())
    for (size_t l = 0; l + 1 < H.levels.size(); ++l)
      build_gs_order(H.levels[l], l > 0, d, prm.color_blocks);
  mark("cells+colours");
  if (prm.settle && coarsest.A.val.size() != coarsest.A.col.size() * static_cast<size_t>(d * d))
    prm.settle(prm.galerkin_ctx);   // a fine level that is also the coarsest: its values now
  dense_cholesky(coarsest.A, coarsest.fixed, H.chol, H.n_coarse_dofs);
  mark("coarsest factor");
}

}  // namespace vasmg

namespace vasmg {
// OpenMP threads of the parallel regions the calling thread starts (setups
// running side by side in a server each get their share of the cores).
void set_host_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
// The calling thread's default OpenMP team size (OMP_NUM_THREADS, else the cores).
int host_thread_budget() { return omp_get_max_threads(); }
}  // namespace vasmg

namespace vasmg {

// Inverse of every vertex's d x d diagonal block (Gauss-Jordan with partial
// pivoting, FP64), [n][d][d] in canonical order.
void block_diag_inverse(const BlockCSR& A, const std::vector<uint8_t>& fixed,
                        std::vector<double>& out) {
  const int d = A.d, dd = d * d;
  const int64_t n = A.n;
  out.assign(static_cast<size_t>(n) * dd, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double a[9], inv[9];
    for (int e = 0; e < dd; ++e) a[e] = 0.0;
    for (int64_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p)
      if (A.col[p] == i)
        for (int e = 0; e < dd; ++e) a[e] = A.val[p * dd + e];
    if (!fixed.empty())   // identity rows of the constrained components
      for (int r = 0; r < d; ++r)
        if ((fixed[i] >> r) & 1) a[r * d + r] = 1.0;
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c) inv[r * d + c] = (r == c) ? 1.0 : 0.0;
    for (int c = 0; c < d; ++c) {
      int piv = c;
      for (int r = c + 1; r < d; ++r)
        if (std::fabs(a[r * d + c]) > std::fabs(a[piv * d + c])) piv = r;
      if (piv != c)
        for (int k = 0; k < d; ++k) {
          std::swap(a[c * d + k], a[piv * d + k]);
          std::swap(inv[c * d + k], inv[piv * d + k]);
        }
      const double pv = a[c * d + c];
      for (int k = 0; k < d; ++k) {
        a[c * d + k] /= pv;
        inv[c * d + k] /= pv;
      }
      for (int r = 0; r < d; ++r) {
        if (r == c) continue;
        const double f = a[r * d + c];
        for (int k = 0; k < d; ++k) {
          a[r * d + k] -= f * a[c * d + k];
          inv[r * d + k] -= f * inv[c * d + k];
        }
      }
    }
    for (int e = 0; e < dd; ++e) out[static_cast<size_t>(i) * dd + e] = inv[e];
  }
}

// Largest eigenvalue of D^{-1} A (D = the vertex blocks): power iteration from
// the all-ones vector, then the Rayleigh quotient v^T A v / v^T D v (FP64).
double jacobi_lambda_max(const BlockCSR& A, const std::vector<double>& dinv, int iters) {
  const int d = A.d, dd = d * d;
  const int64_t n = A.n, N = n * d;
  std::vector<double> v(N, 1.0), w(N), y(N);
  auto apply_A = [&](const std::vector<double>& x, std::vector<double>& out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double acc[3] = {0.0, 0.0, 0.0};
      for (int64_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) {
        const int64_t j = A.col[p];
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b) acc[a] += A.val[p * dd + a * d + b] * x[j * d + b];
      }
      for (int a = 0; a < d; ++a) out[i * d + a] = acc[a];
    }
  };
  for (int it = 0; it < iters; ++it) {
    apply_A(v, y);
    double nrm = 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int a = 0; a < d; ++a) {
        double t = 0.0;
        for (int b = 0; b < d; ++b) t += dinv[i * dd + a * d + b] * y[i * d + b];
        w[i * d + a] = t;
        nrm += t * t;
      }
    nrm = std::sqrt(nrm);
    for (int64_t k = 0; k < N; ++k) v[k] = w[k] / nrm;
  }
  apply_A(v, y);
  double num = 0.0, den = 0.0;
  for (int64_t k = 0; k < N; ++k) num += v[k] * y[k];
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p)
      if (A.col[p] == i)
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b) den += v[i * d + a] * A.val[p * dd + a * d + b] * v[i * d + b];
  return num / den;
}

}  // namespace vasmg

