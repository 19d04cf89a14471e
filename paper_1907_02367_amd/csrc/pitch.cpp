// Advancing-front tent pitcher (Sec. 2.2).
//
// Tents are stacked over vertex patches so that every face stays below the
// characteristic slope 1/c; tents that do not sit on each other are
// independent and are grouped into layers.  The paper delegates the algorithm
// to its reference [MTP] and says the heights are limited by the slopes of
// the mesh edges (Sec. 6).  This file implements that rule:
//   kappa_VW = (gamma * |X_W - X_V|) / c_VW, c_VW = largest speed on edge VW;
//   each layer = local minima of the front (tau_V < T, tau_V <= tau_W for all
//   neighbours W) in (tau_V, V) order, greedily skipping vertices adjacent to
//   one already taken; each is raised to min(T, min_W tau_W + kappa_VW)
//   computed from the front before the layer.
// Afterwards every element of the new tents must satisfy c|grad phi| < 1
// (space-like faces, Sec. 2.2), else TDG_ENONCAUSAL.
//
// Built with -ffp-contract=off: each operation is one IEEE double operation
// in the order written, so the tent list is reproducible bit for bit by any
// implementation that follows the same rule.
#include <algorithm>
#include <cmath>

#include "tdg_internal.h"

namespace tdg {

int pitch_tents(const Topology& topo, double T, double gamma, TentList& out, std::string& err) {
  if (!(T > 0.0) || !std::isfinite(T)) {
    err = "final time T must be positive";
    return TDG_EINVAL;
  }
  if (!(gamma > 0.0) || !std::isfinite(gamma)) {
    err = "gamma must be positive";
    return TDG_EINVAL;
  }
  const int n = topo.n, nv = topo.nv;
  // c_VW and kappa_VW aligned with the neighbour lists
  std::vector<double> kappa(topo.nb.size());
  for (int v = 0; v < nv; ++v) {
    for (int i = topo.nb_ptr[v]; i < topo.nb_ptr[v + 1]; ++i) {
      int w = topo.nb[i];
      double cvw = 0.0;
      for (int j = topo.v2e_ptr[v]; j < topo.v2e_ptr[v + 1]; ++j) {
        int e = topo.v2e[j];
        bool has = false;
        for (int k = 0; k <= n; ++k) has = has || topo.elems[(size_t)e * (n + 1) + k] == w;
        if (has && topo.c[e] > cvw) cvw = topo.c[e];
      }
      double s = 0.0;
      for (int d = 0; d < n; ++d) {
        double diff = topo.coords[(size_t)w * n + d] - topo.coords[(size_t)v * n + d];
        double sq = diff * diff;
        s = s + sq;
      }
      double length = std::sqrt(s);
      double num = gamma * length;
      kappa[i] = num / cvw;
    }
  }
  std::vector<double> tau(nv, 0.0);
  std::vector<int> R, S, stamp(nv, -1);
  std::vector<double> tops;
  out = TentList();
  out.n = n;
  out.T = T;
  out.gamma = gamma;
  out.layer_ptr.push_back(0);
  double max_slope = 0.0;
  for (int layer = 0;; ++layer) {
    R.clear();
    for (int v = 0; v < nv; ++v) {
      if (!(tau[v] < T)) continue;
      bool minimum = true;
      for (int i = topo.nb_ptr[v]; i < topo.nb_ptr[v + 1] && minimum; ++i) minimum = tau[v] <= tau[topo.nb[i]];
      if (minimum) R.push_back(v);
    }
    if (R.empty()) break;
    std::sort(R.begin(), R.end(), [&](int a, int b) { return tau[a] < tau[b] || (tau[a] == tau[b] && a < b); });
    S.clear();
    for (int v : R) {
      bool free = true;
      for (int i = topo.nb_ptr[v]; i < topo.nb_ptr[v + 1] && free; ++i) free = stamp[topo.nb[i]] != layer;
      if (free) {
        S.push_back(v);
        stamp[v] = layer;
      }
    }
    tops.assign(S.size(), 0.0);
    for (size_t s = 0; s < S.size(); ++s) {
      int v = S[s];
      double m = T;
      for (int i = topo.nb_ptr[v]; i < topo.nb_ptr[v + 1]; ++i) {
        double cand = tau[topo.nb[i]] + kappa[i];
        if (cand < m) m = cand;
      }
      tops[s] = m;
    }
    for (size_t s = 0; s < S.size(); ++s) {
      out.V.push_back(S[s]);
      out.tb.push_back(tau[S[s]]);
      out.tt.push_back(tops[s]);
    }
    for (size_t s = 0; s < S.size(); ++s) tau[S[s]] = tops[s];
    // causality of every element under the new tents
    for (int v : S) {
      for (int j = topo.v2e_ptr[v]; j < topo.v2e_ptr[v + 1]; ++j) {
        int e = topo.v2e[j];
        double g[3] = {0, 0, 0};
        for (int k = 0; k <= n; ++k) {
          double tk = tau[topo.elems[(size_t)e * (n + 1) + k]];
          for (int d = 0; d < n; ++d) g[d] = g[d] + tk * topo.grad_lam[((size_t)e * (n + 1) + k) * n + d];
        }
        double g2 = 0.0;
        for (int d = 0; d < n; ++d) g2 = g2 + g[d] * g[d];
        double slope = topo.c[e] * std::sqrt(g2);
        if (slope > max_slope) max_slope = slope;
        if (!(slope < 1.0)) {
          err = "pitched front is not space-like (c|grad phi| >= 1) on element " + std::to_string(e) +
                "; lower gamma";
          return TDG_ENONCAUSAL;
        }
      }
    }
    out.layer_ptr.push_back((int64_t)out.V.size());
  }
  out.max_slope = max_slope;
  return TDG_OK;
}

}  // namespace tdg
