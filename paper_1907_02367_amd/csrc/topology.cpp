// Spatial mesh topology for tent pitching.
//
// A tent at vertex V stands on the vertex patch of V, the elements containing
// V (Sec. 2.2).  Time-like faces inside a tent only sit above facets that
// contain V: facets on the domain boundary (Dirichlet faces of eq. 4.1) and
// facets between two patch elements of different wave speed (Sec. 4.2).
#include <algorithm>
#include <array>
#include <cmath>
#include <map>

#include "tdg_internal.h"

namespace tdg {

namespace {

// Inverts the n x n matrix J (row-major); returns det(J).
double invert_small(int n, const double* J, double* Ji) {
  if (n == 1) {
    Ji[0] = 1.0 / J[0];
    return J[0];
  }
  if (n == 2) {
    double det = J[0] * J[3] - J[1] * J[2];
    Ji[0] = J[3] / det;
    Ji[1] = -J[1] / det;
    Ji[2] = -J[2] / det;
    Ji[3] = J[0] / det;
    return det;
  }
  // n == 3: adjugate
  double a = J[0], b = J[1], c = J[2], d = J[3], e = J[4], f = J[5], g = J[6], h = J[7], i = J[8];
  double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
  double det = a * A + b * B + c * C;
  Ji[0] = A / det;
  Ji[3] = B / det;
  Ji[6] = C / det;
  Ji[1] = -(b * i - c * h) / det;
  Ji[4] = (a * i - c * g) / det;
  Ji[7] = -(a * h - b * g) / det;
  Ji[2] = (b * f - c * e) / det;
  Ji[5] = -(a * f - c * d) / det;
  Ji[8] = (a * e - b * d) / det;
  return det;
}

}  // namespace

int build_topology(const tdg_mesh& m, const double* c, Topology& T, std::string& err) {
  const int n = m.dim;
  if (n < 1 || n > 3) {
    err = "dim must be 1, 2 or 3";
    return TDG_EINVAL;
  }
  if (m.nv <= n || m.ne <= 0 || !m.coords || !m.elems || !c) {
    err = "empty mesh or NULL array";
    return TDG_EINVAL;
  }
  T.n = n;
  T.nv = m.nv;
  T.ne = m.ne;
  T.coords.assign(m.coords, m.coords + (size_t)m.nv * n);
  T.elems.assign(m.elems, m.elems + (size_t)m.ne * (n + 1));
  T.c.assign(c, c + m.ne);
  for (double x : T.coords)
    if (!std::isfinite(x)) {
      err = "non-finite vertex coordinate";
      return TDG_ENAN;
    }
  for (int e = 0; e < m.ne; ++e) {
    if (!(T.c[e] > 0.0) || !std::isfinite(T.c[e])) {
      err = "wave speed must be positive and finite";
      return TDG_EINVAL;
    }
    for (int k = 0; k <= n; ++k) {
      int v = T.elems[(size_t)e * (n + 1) + k];
      if (v < 0 || v >= m.nv) {
        err = "element vertex index out of range";
        return TDG_EINVAL;
      }
      for (int l = 0; l < k; ++l)
        if (T.elems[(size_t)e * (n + 1) + l] == v) {
          err = "element with a repeated vertex";
          return TDG_EINVAL;
        }
    }
  }
  // patches (ascending element index)
  T.v2e_ptr.assign(m.nv + 1, 0);
  for (int e = 0; e < m.ne; ++e)
    for (int k = 0; k <= n; ++k) T.v2e_ptr[T.elems[(size_t)e * (n + 1) + k] + 1]++;
  for (int v = 0; v < m.nv; ++v) T.v2e_ptr[v + 1] += T.v2e_ptr[v];
  T.v2e.assign(T.v2e_ptr[m.nv], 0);
  {
    std::vector<int> fill(T.v2e_ptr.begin(), T.v2e_ptr.end() - 1);
    for (int e = 0; e < m.ne; ++e)
      for (int k = 0; k <= n; ++k) T.v2e[fill[T.elems[(size_t)e * (n + 1) + k]]++] = e;
  }
  for (int v = 0; v < m.nv; ++v) {
    int cnt = T.v2e_ptr[v + 1] - T.v2e_ptr[v];
    if (cnt == 0) {
      err = "vertex not used by any element";
      return TDG_EINVAL;
    }
    if (cnt > kMaxPatch) {
      err = "vertex patch larger than the supported maximum";
      return TDG_EINVAL;
    }
  }
  // neighbours (ascending)
  T.nb_ptr.assign(m.nv + 1, 0);
  std::vector<std::vector<int>> nb(m.nv);
  for (int v = 0; v < m.nv; ++v) {
    auto& s = nb[v];
    for (int i = T.v2e_ptr[v]; i < T.v2e_ptr[v + 1]; ++i) {
      int e = T.v2e[i];
      for (int k = 0; k <= n; ++k) {
        int w = T.elems[(size_t)e * (n + 1) + k];
        if (w != v) s.push_back(w);
      }
    }
    std::sort(s.begin(), s.end());
    s.erase(std::unique(s.begin(), s.end()), s.end());
    T.nb_ptr[v + 1] = T.nb_ptr[v] + (int)s.size();
  }
  T.nb.reserve(T.nb_ptr[m.nv]);
  for (int v = 0; v < m.nv; ++v) T.nb.insert(T.nb.end(), nb[v].begin(), nb[v].end());
  // barycentric gradients and |det|
  T.grad_lam.assign((size_t)m.ne * (n + 1) * n, 0.0);
  T.absdet.assign(m.ne, 0.0);
  for (int e = 0; e < m.ne; ++e) {
    const int* vs = &T.elems[(size_t)e * (n + 1)];
    double J[9], Ji[9];
    double scale = 0.0;
    for (int r = 0; r < n; ++r)
      for (int k = 1; k <= n; ++k) {
        // J[r][k-1] = X_k[r] - X_0[r]  (columns are edge vectors)
        J[r * n + (k - 1)] = T.coords[(size_t)vs[k] * n + r] - T.coords[(size_t)vs[0] * n + r];
        scale = std::max(scale, std::fabs(J[r * n + (k - 1)]));
      }
    double det = invert_small(n, J, Ji);
    if (!(std::fabs(det) > 1e-13 * std::pow(scale, n))) {
      err = "degenerate element (zero volume)";
      return TDG_EINVAL;
    }
    T.absdet[e] = std::fabs(det);
    double* g = &T.grad_lam[(size_t)e * (n + 1) * n];
    for (int d = 0; d < n; ++d) g[d] = 0.0;
    for (int k = 1; k <= n; ++k)
      for (int d = 0; d < n; ++d) {
        // grad lambda_k = row k-1 of J^{-1}
        g[k * n + d] = Ji[(k - 1) * n + d];
        g[d] -= Ji[(k - 1) * n + d];
      }
  }
  // facets: sorted vertex tuple -> (element, opposite local vertex), elements ascending
  std::map<std::array<int, 3>, std::vector<std::pair<int, int>>> facets;
  for (int e = 0; e < m.ne; ++e) {
    const int* vs = &T.elems[(size_t)e * (n + 1)];
    for (int k = 0; k <= n; ++k) {
      std::array<int, 3> key{-1, -1, -1};
      int j = 0;
      for (int l = 0; l <= n; ++l)
        if (l != k) key[j++] = vs[l];
      std::sort(key.begin(), key.begin() + n);
      facets[key].push_back({e, k});
    }
  }
  auto facet_key = [&](int e, int k) {
    const int* vs = &T.elems[(size_t)e * (n + 1)];
    std::array<int, 3> key{-1, -1, -1};
    int j = 0;
    for (int l = 0; l <= n; ++l)
      if (l != k) key[j++] = vs[l];
    std::sort(key.begin(), key.begin() + n);
    return key;
  };
  for (auto& kv : facets)
    if (kv.second.size() > 2) {
      err = "non-manifold mesh: a facet shared by more than two elements";
      return TDG_EINVAL;
    }
  // boundary facets in ascending (element, opposite local vertex) order: the
  // order of the per-facet kinds of tdg_mesh.bface_kind
  T.bfacets.clear();
  for (auto& kv : facets)
    if (kv.second.size() == 1) T.bfacets.push_back(kv.second[0]);
  std::sort(T.bfacets.begin(), T.bfacets.end());
  std::map<std::pair<int, int>, int> bkind;
  for (size_t i = 0; i < T.bfacets.size(); ++i) {
    const int kd = m.bface_kind ? (int)m.bface_kind[i] : 0;
    if (kd != 0 && kd != 1) {
      err = "bface_kind entries must be 0 (Dirichlet) or 1 (Neumann)";
      return TDG_EINVAL;
    }
    bkind[T.bfacets[i]] = kd;
  }
  T.vb_ptr.assign(m.nv + 1, 0);
  T.vn_ptr.assign(m.nv + 1, 0);
  T.vi_ptr.assign(m.nv + 1, 0);
  T.vb.clear();
  T.vn.clear();
  T.vi.clear();
  for (int v = 0; v < m.nv; ++v) {
    std::vector<std::array<int, 4>> inter;
    for (int i = T.v2e_ptr[v]; i < T.v2e_ptr[v + 1]; ++i) {
      int e = T.v2e[i];
      for (int k = 0; k <= n; ++k) {
        if (T.elems[(size_t)e * (n + 1) + k] == v) continue;
        const auto& sides = facets[facet_key(e, k)];
        if (sides.size() == 1) {
          std::vector<int>& dst = bkind[{e, k}] == 0 ? T.vb : T.vn;
          dst.push_back(e);
          dst.push_back(k);
        } else if (sides[0].first == e && T.c[sides[0].first] != T.c[sides[1].first]) {
          inter.push_back({sides[0].first, sides[0].second, sides[1].first, sides[1].second});
        }
      }
    }
    std::sort(inter.begin(), inter.end());
    for (auto& q : inter) T.vi.insert(T.vi.end(), q.begin(), q.end());
    T.vb_ptr[v + 1] = (int)T.vb.size() / 2;
    T.vn_ptr[v + 1] = (int)T.vn.size() / 2;
    T.vi_ptr[v + 1] = (int)T.vi.size() / 4;
  }
  return TDG_OK;
}

}  // namespace tdg
