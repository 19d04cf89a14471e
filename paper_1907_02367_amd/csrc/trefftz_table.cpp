// Exact Trefftz basis tables of U^p (Sec. 3).
//
// U(x,t) = sum_{k+|alpha|<=p} a_{k,alpha} x^alpha t^k solves -Lap U + U_tt = 0
// (c = 1) iff for k >= 2
//   a_{k,alpha} = 1/(k(k-1)) sum_m (alpha_m+1)(alpha_m+2) a_{k-2,alpha+2e_m}   (eq. 3.1)
// seeded by a basis of the spatial polynomials: U(.,0) = b_beta, U_t(.,0) = 0
// for |beta| <= p, then U(.,0) = 0, U_t(.,0) = b_beta for |beta| <= p-1
// (dim = C(p+n,n) + C(p-1+n,n)).  b_beta is the monomial x^beta (seed 0), or
// the product over the variables of Legendre polynomials P_(beta_m)(x_m)
// (seed 1) or Chebyshev polynomials T_(beta_m)(x_m) (seed 2), the three
// choices of Sec. 6.3; the recursion is linear in the seed, so a seeded
// function is the same combination of the monomial-seeded ones.
// Any c is reached by the change of variables of Remark 3.1, applied in the
// kernels.  Coefficients are computed in exact 64-bit rationals (they stay
// far below 2^53 for p <= 10) and rounded once to double.
//
// Basis order: seed type 0 then type 1, each by |beta| ascending then beta in
// descending lexicographic order; function 0 is the constant.  The tables
// hold the first-order fields (v, sigma) = (dU/dt, -grad U) of functions
// 1..N-1 and the functions themselves (to recover U, Sec. 5).
#include <algorithm>
#include <array>
#include <map>
#include <numeric>
#include <stdexcept>

#include "trefftz_table.h"

namespace tdg {

namespace {

struct Rat {
  int64_t num = 0, den = 1;
  Rat() = default;
  Rat(int64_t a, int64_t b = 1) : num(a), den(b) { norm(); }
  void norm() {
    if (den < 0) {
      num = -num;
      den = -den;
    }
    int64_t g = std::gcd(num < 0 ? -num : num, den);
    if (g > 1) {
      num /= g;
      den /= g;
    }
    if (num == 0) den = 1;
  }
  static int64_t fit(__int128 v) {
    if (v > (__int128)INT64_MAX || v < -(__int128)INT64_MAX) throw std::overflow_error("Trefftz table coefficient overflow");
    return (int64_t)v;
  }
  Rat operator+(const Rat& o) const {
    __int128 n = (__int128)num * o.den + (__int128)o.num * den;
    __int128 d = (__int128)den * o.den;
    __int128 a = n < 0 ? -n : n, b = d, t;
    while (b) {
      t = a % b;
      a = b;
      b = t;
    }
    if (a > 1) {
      n /= a;
      d /= a;
    }
    Rat r;
    r.num = fit(n);
    r.den = fit(d);
    r.norm();
    return r;
  }
  Rat mul(int64_t k) const { return Rat(fit((__int128)num * k), den); }
  Rat div(int64_t k) const { return Rat(num, fit((__int128)den * k)); }
  Rat mul(const Rat& o) const {
    // cross-reduce first so the products stay small
    const int64_t g1 = std::gcd(num < 0 ? -num : num, o.den), g2 = std::gcd(o.num < 0 ? -o.num : o.num, den);
    const int64_t a = g1 ? num / g1 : num, b = g2 ? o.num / g2 : o.num;
    const int64_t c = g2 ? den / g2 : den, d = g1 ? o.den / g1 : o.den;
    return Rat(fit((__int128)a * b), fit((__int128)c * d));
  }
  double to_double() const { return (double)num / (double)den; }
  bool zero() const { return num == 0; }
};

using Key = std::array<int, 4>;  // k, alpha_1..alpha_3 (unused entries 0)

// multi-indices of length n with |alpha| = deg, descending lexicographic order
std::vector<Key> multi(int n, int deg) {
  std::vector<Key> out;
  Key a{0, 0, 0, 0};
  // enumerate all with entries in [0, deg]
  int total = 1;
  for (int i = 0; i < n; ++i) total *= (deg + 1);
  for (int idx = 0; idx < total; ++idx) {
    int r = idx, s = 0;
    Key al{0, 0, 0, 0};
    for (int i = n - 1; i >= 0; --i) {
      al[1 + i] = r % (deg + 1);
      r /= (deg + 1);
      s += al[1 + i];
    }
    if (s == deg) out.push_back(al);
  }
  std::sort(out.begin(), out.end(), [](const Key& x, const Key& y) { return x > y; });
  (void)a;
  return out;
}

// Coefficients c_0..c_d of the degree-d seed polynomial of one variable, from
// the closed forms (Sec. 6.3 names the families):
//   Legendre  P_d(x) = 2^-d sum_k (-1)^k C(d,k) C(2d-2k,d) x^(d-2k),
//   Chebyshev T_d(x) = sum_k (-1)^k d 2^(d-2k-1) (d-k-1)! / (k! (d-2k)!) x^(d-2k)  (d >= 1).
std::vector<Rat> seed_1d(int kind, int d) {
  std::vector<Rat> c((size_t)d + 1, Rat(0));
  auto binom = [](int a, int b) {
    int64_t r = 1;
    for (int i = 1; i <= b; ++i) r = r * (a - b + i) / i;
    return r;
  };
  auto fact = [](int a) {
    int64_t r = 1;
    for (int i = 2; i <= a; ++i) r *= i;
    return r;
  };
  if (kind == 0 || d == 0) {
    c[(size_t)d] = Rat(1);
    return c;
  }
  for (int k = 0; 2 * k <= d; ++k) {
    const int64_t sg = (k & 1) ? -1 : 1;
    if (kind == 1)
      c[(size_t)(d - 2 * k)] = Rat(sg * binom(d, k) * binom(2 * d - 2 * k, d), (int64_t)1 << d);
    else
      c[(size_t)(d - 2 * k)] =
          Rat(sg * d * fact(d - k - 1), fact(k) * fact(d - 2 * k)).mul((int64_t)1 << (d - 2 * k)).div(2);
  }
  return c;
}

}  // namespace

Table build_table(int n, int p, int seed) {
  if (seed < 0 || seed > 2) throw std::invalid_argument("seed basis must be 0, 1 or 2");
  Table T;
  T.n = n;
  T.p = p;
  // monomials by total degree; inside a degree: k descending, alpha descending lex
  std::map<Key, int> index;
  std::vector<Key> mono;
  for (int d = 0; d <= p; ++d) {
    for (int k = d; k >= 0; --k)
      for (Key al : multi(n, d - k)) {
        al[0] = k;
        index[al] = (int)mono.size();
        mono.push_back(al);
      }
    if (d == p - 1) T.M1 = (int)mono.size();
  }
  if (p == 0) T.M1 = 0;
  T.M = (int)mono.size();
  T.parent.assign(T.M, -1);
  T.var.assign(T.M, 0);
  T.expo.assign((size_t)T.M * (n + 1), 0);
  for (int i = 0; i < T.M; ++i) {
    Key m = mono[i];
    for (int j = 0; j <= n; ++j) T.expo[(size_t)i * (n + 1) + j] = m[j];
    if (i == 0) continue;
    Key par = m;
    if (m[0] > 0) {
      par[0]--;
      T.var[i] = 0;
    } else {
      int j = 1;
      while (m[j] == 0) ++j;
      par[j]--;
      T.var[i] = j;
    }
    T.parent[i] = index.at(par);
  }
  // basis functions
  std::vector<std::pair<int, Key>> seeds;
  for (int d = 0; d <= p; ++d)
    for (Key b : multi(n, d)) seeds.push_back({0, b});
  for (int d = 0; d + 1 <= p; ++d)
    for (Key b : multi(n, d)) seeds.push_back({1, b});
  std::vector<std::map<Key, Rat>> basis;
  for (auto& sd : seeds) {
    std::map<Key, Rat> a;
    Key s = sd.second;
    s[0] = sd.first;
    a[s] = Rat(1);
    for (int k = 2; k <= p; ++k)
      for (int d = 0; d <= p - k; ++d)
        for (Key al : multi(n, d)) {
          Rat acc;
          for (int m = 0; m < n; ++m) {
            Key up = al;
            up[0] = k - 2;
            up[1 + m] += 2;
            auto it = a.find(up);
            if (it != a.end() && !it->second.zero())
              acc = acc + it->second.mul((int64_t)(al[1 + m] + 1) * (al[1 + m] + 2));
          }
          if (!acc.zero()) {
            Key key = al;
            key[0] = k;
            a[key] = acc.div((int64_t)k * (k - 1));
          }
        }
    basis.push_back(a);
  }
  if (seed != 0) {
    // b_beta = sum_gamma prod_m s_(beta_m)[gamma_m] x^gamma: combine the
    // monomial-seeded functions of the same type with those weights
    std::map<std::pair<int, Key>, int> pos;
    for (size_t i = 0; i < seeds.size(); ++i) pos[seeds[i]] = (int)i;
    std::vector<std::map<Key, Rat>> comb(seeds.size());
    for (size_t i = 0; i < seeds.size(); ++i) {
      const Key b = seeds[i].second;
      std::vector<std::vector<Rat>> s1(n);
      for (int m = 0; m < n; ++m) s1[m] = seed_1d(seed, b[1 + m]);
      Key g{0, 0, 0, 0};
      // every gamma with gamma_m <= beta_m
      for (;;) {
        Rat w(1);
        for (int m = 0; m < n; ++m) w = w.mul(s1[m][(size_t)g[1 + m]]);
        if (!w.zero())
          for (auto& kv : basis[(size_t)pos.at({seeds[i].first, g})]) {
            Rat& dst = comb[i][kv.first];
            dst = dst + kv.second.mul(w);
          }
        int m = 0;
        while (m < n && g[1 + m] == b[1 + m]) g[1 + m++] = 0;
        if (m == n) break;
        g[1 + m]++;
      }
      for (auto it = comb[i].begin(); it != comb[i].end();) it = it->second.zero() ? comb[i].erase(it) : std::next(it);
    }
    basis.swap(comb);
  }
  const int N = (int)basis.size();
  T.NW = N - 1;
  // first-order fields: rows j*(n+1)+comp
  T.fo_ptr.assign((size_t)T.NW * (n + 1) + 1, 0);
  T.u_ptr.assign((size_t)T.NW + 1, 0);
  for (int j = 0; j < T.NW; ++j) {
    const auto& b = basis[j + 1];
    for (int comp = 0; comp <= n; ++comp) {
      std::map<int, Rat> row;
      for (auto& kv : b) {
        Key key = kv.first;
        if (comp == 0) {
          if (key[0] == 0) continue;
          Rat v = kv.second.mul(key[0]);
          key[0]--;
          row[index.at(key)] = row[index.at(key)] + v;
        } else {
          int al = key[comp];
          if (al == 0) continue;
          Rat v = kv.second.mul(-al);
          key[comp]--;
          row[index.at(key)] = row[index.at(key)] + v;
        }
      }
      for (auto& kv : row)
        if (!kv.second.zero()) {
          T.fo_idx.push_back(kv.first);
          T.fo_coef.push_back(kv.second.to_double());
        }
      T.fo_ptr[(size_t)j * (n + 1) + comp + 1] = (int)T.fo_idx.size();
    }
    std::map<int, Rat> urow;
    for (auto& kv : b) urow[index.at(kv.first)] = kv.second;
    for (auto& kv : urow)
      if (!kv.second.zero()) {
        T.u_idx.push_back(kv.first);
        T.u_coef.push_back(kv.second.to_double());
      }
    T.u_ptr[j + 1] = (int)T.u_idx.size();
  }
  // entry form: one entry per term a x^alpha t^k of U_j, with the derivative terms
  // k a x^alpha t^(k-1) (v) and -alpha_m a x^(alpha-e_m) t^k (sigma_m)
  const int ns = n + 2;
  T.ue_ptr.assign((size_t)T.NW + 1, 0);
  for (int j = 0; j < T.NW; ++j) {
    for (auto& kv : basis[j + 1]) {
      const Key key = kv.first;
      const Rat a = kv.second;
      T.ue_idx.push_back(index.at(key));
      T.ue_coef.push_back(a.to_double());
      if (key[0] > 0) {
        Key d = key;
        d[0]--;
        T.ue_idx.push_back(index.at(d));
        T.ue_coef.push_back(a.mul(key[0]).to_double());
      } else {
        T.ue_idx.push_back(0);
        T.ue_coef.push_back(0.0);
      }
      for (int m = 1; m <= n; ++m) {
        if (key[m] > 0) {
          Key d = key;
          d[m]--;
          T.ue_idx.push_back(index.at(d));
          T.ue_coef.push_back(a.mul(-key[m]).to_double());
        } else {
          T.ue_idx.push_back(0);
          T.ue_coef.push_back(0.0);
        }
      }
    }
    T.ue_ptr[j + 1] = (int)(T.ue_idx.size() / ns);
  }
  // moment monomials (degree <= 2p-2, same order convention) and the index of
  // the product of monomials k, l < M1 among them: the Gram of the fields is a
  // combination of the moments of these products over the points
  {
    const int d2 = std::max(2 * p - 2, 0);
    std::map<Key, int> index2;
    for (int d = 0; d <= d2; ++d)
      for (int k = d; k >= 0; --k)
        for (Key al : multi(n, d - k)) {
          al[0] = k;
          index2[al] = (int)(T.expo2.size() / (n + 1));
          for (int j = 0; j <= n; ++j) T.expo2.push_back(al[j]);
        }
    T.M2 = (int)(T.expo2.size() / (n + 1));
    T.K2.assign((size_t)T.M1 * T.M1, 0);
    for (int a = 0; a < T.M1; ++a)
      for (int b = 0; b < T.M1; ++b) {
        Key sum{0, 0, 0, 0};
        for (int j = 0; j <= n; ++j) sum[j] = mono[a][j] + mono[b][j];
        T.K2[(size_t)a * T.M1 + b] = index2.at(sum);
      }
  }
  // moment tasks: monomials sharing all exponents but the last, in runs of up to
  // four consecutive last exponents (a thread forms the shared prefix once and
  // steps the last variable), for the moment list (degree <= 2p-2) and for the
  // monomials of degree <= p
  auto tasks = [&](const std::vector<int>& ex, int count, std::vector<int>& out) {
    std::map<std::array<int, 3>, std::vector<std::pair<int, int>>> runs;  // prefix -> (last exponent, index)
    for (int i = 0; i < count; ++i) {
      std::array<int, 3> pre{0, 0, 0};
      for (int j = 0; j < n; ++j) pre[j] = ex[(size_t)i * (n + 1) + j];
      runs[pre].push_back({ex[(size_t)i * (n + 1) + n], i});
    }
    for (auto& kv : runs) {
      auto& v = kv.second;
      std::sort(v.begin(), v.end());
      for (size_t a = 0; a < v.size(); a += 4) {
        const int cnt = (int)std::min<size_t>(4, v.size() - a);
        // the run has consecutive last exponents
        for (int c = 1; c < cnt; ++c)
          if (v[a + c].first != v[a].first + c) throw std::runtime_error("moment run with a gap");
        int idx[4];
        for (int c = 0; c < 4; ++c) idx[c] = c < cnt ? v[a + c].second : 0xFFFF;
        for (int c = 0; c < cnt; ++c)
          if (idx[c] >= 0xFFFF) throw std::runtime_error("moment index beyond 16 bits");
        const unsigned w0 = (unsigned)kv.first[0] | (unsigned)kv.first[1] << 5 | (unsigned)kv.first[2] << 10 |
                            (unsigned)v[a].first << 15;
        out.push_back((int)w0);
        out.push_back((int)((unsigned)idx[0] | (unsigned)idx[1] << 16));
        out.push_back((int)((unsigned)idx[2] | (unsigned)idx[3] << 16));
      }
    }
  };
  tasks(T.expo2, T.M2, T.task2);
  T.ntask2 = (int)(T.task2.size() / kTaskInts);
  // matrix-core tiles of the top moments (3+1D): L = t^a0 x1^a1 and
  // R = x2^c0 x3^c1, each list of degree <= D = 2p-2 ordered by degree, so a
  // 16-row block of L and a 16-column block of R hold a product of degree <= D
  // only if their smallest degrees add up to at most D; the moment index of
  // every such product (or -1 past D or past the lists) is tabulated
  if (n == 3 && p >= 2) {
    const int D = 2 * p - 2;
    std::vector<std::array<int, 2>> Ls, Rs;
    for (int d = 0; d <= D; ++d)
      for (int a = d; a >= 0; --a) Ls.push_back({a, d - a});
    Rs = Ls;
    const int nI = ((int)Ls.size() + 15) / 16, nJ = ((int)Rs.size() + 15) / 16;
    auto deg = [](const std::array<int, 2>& e) { return e[0] + e[1]; };
    std::map<Key, int> index2;
    for (int i = 0; i < T.M2; ++i) {
      Key k{0, 0, 0, 0};
      for (int j = 0; j <= n; ++j) k[j] = T.expo2[(size_t)i * (n + 1) + j];
      index2[k] = i;
    }
    std::vector<std::array<int, 2>> tiles;
    for (int I = 0; I < nI; ++I)
      for (int J = 0; J < nJ; ++J)
        if (deg(Ls[16 * I]) + deg(Rs[16 * J]) <= D) tiles.push_back({I, J});
    if ((int)tiles.size() <= 4 * kMomTileSlots) {
      T.mt_ntile = (int)tiles.size();
      std::vector<int> seen((size_t)T.M2, 0);
      for (auto& tj : tiles) {
        for (int l = 0; l < 16; ++l) {
          const int i = 16 * tj[0] + l, j = 16 * tj[1] + l;
          const std::array<int, 2> a = i < (int)Ls.size() ? Ls[i] : std::array<int, 2>{0, 0};
          const std::array<int, 2> c = j < (int)Rs.size() ? Rs[j] : std::array<int, 2>{0, 0};
          T.mt_ex.push_back(a[0] | a[1] << 5 | c[0] << 10 | c[1] << 15);
        }
        for (int r = 0; r < 16; ++r)
          for (int cc = 0; cc < 16; ++cc) {
            const int i = 16 * tj[0] + r, j = 16 * tj[1] + cc;
            int b = -1;
            if (i < (int)Ls.size() && j < (int)Rs.size() && deg(Ls[i]) + deg(Rs[j]) <= D) {
              b = index2.at(Key{Ls[i][0], Ls[i][1], Rs[j][0], Rs[j][1]});
              seen[(size_t)b]++;
            }
            T.mt_map.push_back(b);
          }
      }
      // every moment monomial is formed exactly once
      for (int i = 0; i < T.M2; ++i)
        if (seen[(size_t)i] != 1) throw std::runtime_error("matrix-core moment tiles do not cover the moments");
    }
  }
  tasks(T.expo, T.M, T.task1);
  T.ntask1 = (int)(T.task1.size() / kTaskInts);
  // matrix-core evaluation (3+1D): every monomial of degree <= p is the product
  // of an entry of the two-variable list (t, x1) and one of (x2, x3), both by
  // degree; a tile of 16 (t, x1)-entries of smallest degree d needs the
  // (x2, x3)-entries of degree <= p - d
  if (n == 3) {
    std::vector<std::array<int, 2>> lst;
    std::map<std::array<int, 2>, int> pos;
    for (int d = 0; d <= p; ++d)
      for (int a = d; a >= 0; --a) {
        pos[{a, d - a}] = (int)lst.size();
        lst.push_back({a, d - a});
      }
    const int nl = (int)lst.size();
    const int nat = (nl + 15) / 16;
    if (nat <= 8 && (nl + 3) / 4 <= kEvalMaxSteps) {
      T.ev_nl = nl;
      T.ev_nat = nat;
      for (auto& e : lst) T.ev_ex.push_back(e[0] | e[1] << 8);
      for (int I = 0; I < nat; ++I) {
        const int dmin = lst[16 * I][0] + lst[16 * I][1];
        const int need = (p - dmin + 1) * (p - dmin + 2) / 2;  // entries of degree <= p - dmin
        T.ev_nks[I] = (need + 3) / 4;
        // v and sigma have degree <= p - 1: entries of degree <= p - 1 - dmin
        const int bv = p - 1 - dmin;
        T.ev_nkv[I] = bv < 0 ? 0 : ((bv + 1) * (bv + 2) / 2 + 3) / 4;
      }
      for (int k = 0; k < T.M; ++k) {
        const int* e = &T.expo[(size_t)k * (n + 1)];
        const int a = pos.at({e[0], e[1]}), b = pos.at({e[2], e[3]});
        T.ev_ab.push_back(a | b << 16);
      }
    }
  }
  // transposed form: rows comp*M + monomial
  {
    std::vector<std::vector<std::pair<int, double>>> rows((size_t)ns * T.M);
    for (int j = 0; j < T.NW; ++j)
      for (int comp = 0; comp <= n; ++comp)
        for (int e = T.fo_ptr[(size_t)j * (n + 1) + comp]; e < T.fo_ptr[(size_t)j * (n + 1) + comp + 1]; ++e)
          rows[(size_t)comp * T.M + T.fo_idx[e]].push_back({j, T.fo_coef[e]});
    for (int j = 0; j < T.NW; ++j)
      for (int e = T.u_ptr[j]; e < T.u_ptr[j + 1]; ++e)
        rows[(size_t)(n + 1) * T.M + T.u_idx[e]].push_back({j, T.u_coef[e]});
    T.tr_ptr.assign(rows.size() + 1, 0);
    for (size_t r = 0; r < rows.size(); ++r) {
      for (auto& pr : rows[r]) {
        T.tr_j.push_back(pr.first);
        T.tr_coef.push_back(pr.second);
      }
      T.tr_ptr[r + 1] = (int)T.tr_j.size();
    }
  }
  return T;
}

// The monomial-seeded tables, the library's default basis.
Table build_table(int n, int p) { return build_table(n, p, 0); }

}  // namespace tdg
