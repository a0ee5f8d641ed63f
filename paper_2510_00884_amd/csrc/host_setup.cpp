// Host-side mesh setup (not on the hot path): CSR sparsity of the global
// stiffness over node-major dofs and a greedy element colouring.
#include <algorithm>
#include <cstdint>
#include <vector>

namespace pa {

// node -> elements adjacency in CSR form
static void node_elements(int nen, int64_t n_el, int64_t n_nodes, const int32_t* conn,
                          std::vector<int64_t>& ptr, std::vector<int32_t>& idx) {
  ptr.assign(n_nodes + 1, 0);
  for (int64_t e = 0; e < n_el; ++e)
    for (int a = 0; a < nen; ++a) ptr[conn[e * nen + a] + 1]++;
  for (int64_t i = 0; i < n_nodes; ++i) ptr[i + 1] += ptr[i];
  idx.resize(ptr[n_nodes]);
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t e = 0; e < n_el; ++e)
    for (int a = 0; a < nen; ++a) idx[fill[conn[e * nen + a]]++] = (int32_t)e;
}

int host_csr_pattern(int nen, int64_t n_el, int64_t n_nodes, const int32_t* conn, int64_t* row_ptr,
                     int32_t* col, int64_t* nnz_out) {
  for (int64_t i = 0; i < n_el * nen; ++i)
    if (conn[i] < 0 || conn[i] >= n_nodes) return -1;
  std::vector<int64_t> eptr;
  std::vector<int32_t> eidx;
  node_elements(nen, n_el, n_nodes, conn, eptr, eidx);
  std::vector<int32_t> nb;
  int64_t nnz = 0;
  if (row_ptr) row_ptr[0] = 0;
  for (int64_t I = 0; I < n_nodes; ++I) {
    nb.clear();
    for (int64_t k = eptr[I]; k < eptr[I + 1]; ++k) {
      const int64_t e = eidx[k];
      for (int a = 0; a < nen; ++a) nb.push_back(conn[e * nen + a]);
    }
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    const int64_t len = 3 * (int64_t)nb.size();
    for (int i = 0; i < 3; ++i) {
      if (col) {
        int32_t* c = col + nnz;
        for (size_t t = 0; t < nb.size(); ++t) {
          c[3 * t] = 3 * nb[t];
          c[3 * t + 1] = 3 * nb[t] + 1;
          c[3 * t + 2] = 3 * nb[t] + 2;
        }
      }
      nnz += len;
      if (row_ptr) row_ptr[3 * I + i + 1] = nnz;
    }
  }
  *nnz_out = nnz;
  return 0;
}

// For every node, the (element, local node) pairs that touch it as e*nen + a,
// in ascending element order (the summation order of the gather assembly).
int host_node_incidence(int nen, int64_t n_el, int64_t n_nodes, const int32_t* conn, int64_t* ptr,
                        int32_t* ent) {
  for (int64_t i = 0; i < n_el * nen; ++i)
    if (conn[i] < 0 || conn[i] >= n_nodes) return -1;
  for (int64_t i = 0; i <= n_nodes; ++i) ptr[i] = 0;
  for (int64_t e = 0; e < n_el; ++e)
    for (int a = 0; a < nen; ++a) ptr[conn[e * nen + a] + 1]++;
  for (int64_t i = 0; i < n_nodes; ++i) ptr[i + 1] += ptr[i];
  if (ent) {
    std::vector<int64_t> fill(ptr, ptr + n_nodes);
    for (int64_t e = 0; e < n_el; ++e)
      for (int a = 0; a < nen; ++a) ent[fill[conn[e * nen + a]]++] = (int32_t)(e * nen + a);
  }
  return 0;
}

int host_colour(int nen, int64_t n_el, int64_t n_nodes, const int32_t* conn, int32_t* colour,
                int32_t* n_colours) {
  for (int64_t i = 0; i < n_el * nen; ++i)
    if (conn[i] < 0 || conn[i] >= n_nodes) return -1;
  std::vector<int64_t> eptr;
  std::vector<int32_t> eidx;
  node_elements(nen, n_el, n_nodes, conn, eptr, eidx);
  std::vector<int64_t> mark;  // mark[c] = last element that saw colour c in use
  int32_t nc = 0;
  for (int64_t e = 0; e < n_el; ++e) colour[e] = -1;
  for (int64_t e = 0; e < n_el; ++e) {
    for (int a = 0; a < nen; ++a) {
      const int64_t I = conn[e * nen + a];
      for (int64_t k = eptr[I]; k < eptr[I + 1]; ++k) {
        const int32_t c = colour[eidx[k]];
        if (c >= 0) mark[c] = e;
      }
    }
    int32_t c = 0;
    while (c < nc && mark[c] == e) ++c;
    if (c == nc) { mark.push_back(-1); ++nc; }
    colour[e] = c;
  }
  *n_colours = nc;
  return 0;
}

}  // namespace pa
