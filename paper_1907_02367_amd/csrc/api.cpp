// C-ABI of libtdg: tent pitching, solver context, buffers, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>

#include "tdg_internal.h"
#include "trefftz_table.h"

namespace tdg {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

}  // namespace tdg

using namespace tdg;

#define TDG_TRY_BEGIN try {
#define TDG_TRY_END                      \
  }                                      \
  catch (const std::bad_alloc&) {        \
    set_error("host allocation failed"); \
    return TDG_ENOMEM;                   \
  }                                      \
  catch (const std::exception& ex) {     \
    set_error(ex.what());                \
    return TDG_EINVAL;                   \
  }

#define HIP_OK(call)                                                                \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " in " #call); \
      return TDG_EHIP;                                                              \
    }                                                                               \
  } while (0)

struct tdg_ctx {
  Topology topo;
  Quadrature quad;
  std::vector<Table> tabs;  // index p (0 unused)
  TentList tents;
  tdg_opts opts{};
  int64_t nq = 0, nb = 0;
  std::vector<int64_t> bpt_off;
  std::vector<double> bpts;  // nb * (n+1)
  std::vector<int8_t> bkind;  // nb: 0 = point of a Dirichlet face (g_D), 1 = of a Neumann face (g_N)
  int max_groups = 1;
  // staged static tables
  std::vector<double> hf64;
  std::vector<int> hi32;
  struct TabOff {
    size_t parent, var, expo, fo_ptr, fo_idx, u_ptr, u_idx, ue_ptr, ue_idx, tr_ptr, tr_j, expo2, K2, task2,
        task1, mt_ex, mt_map, ev_ab, ev_ex;  // i32
    size_t ue_coef, tr_coef;                                                           // f64
    size_t fo_coef, u_coef, fo_coef32;                 // f64 (fo_coef32: floats packed two per double)
  } toff[kMaxP + 1];
  size_t o_coords, o_c, o_grad, o_det, o_lam, o_w, o_tb, o_tt, o_bpt;         // f64
  size_t o_elems, o_v2e_ptr, o_v2e, o_vb_ptr, o_vb, o_vn_ptr, o_vn, o_vi_ptr, o_vi, o_tentV;  // i32
  TableDesc tabd[kMaxP + 1]{};  // per-degree tables and plan, mirrored on the device
  size_t o_tabd = 0;             // offset (doubles) of the device copy in the FP64 buffer
  int gram_mode = 0;   // 0: Gram of the basis values at the points (matrix cores); 1: from moments
  int forced_pch = 0;  // points per chunk set by trefftz_set_tuning (0: largest that fits)
  int64_t sizes[TDG_NBUF]{};
  void* dev[TDG_NBUF]{};
  bool bound = false;
  KParams kp{};
  LdsPlan lp{};
  size_t w_ex = 0, w_partial = 0, w_out = 0, w_status = 0, w_sys = 0, w_ctr = 0;  // offsets in doubles inside WORK
  size_t w_order = 0;  // the layers' queue orders (one int per tent)
  int persistent = 0, ncu = 256, resident = 1;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int64_t sys_stride = 0;  // doubles per workgroup for systems kept in global memory
  int nblocks_red = 256;
};

namespace {

size_t push(std::vector<double>& v, const double* p, size_t n) {
  size_t off = v.size();
  v.insert(v.end(), p, p + n);
  while (v.size() % 32) v.push_back(0.0);  // 256-byte alignment
  return off;
}
size_t push(std::vector<int>& v, const int* p, size_t n) {
  size_t off = v.size();
  v.insert(v.end(), p, p + n);
  while (v.size() % 64) v.push_back(0);
  return off;
}

int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

// element-record size of the tent kernel (see El<NS> in the kernel)
int el_size(int n) { return (n + 1) * n + (n + 1) + 2 * n + 5; }

// Panel width of the blocked LU of a system held in global memory (3+1D
// kernels): the panel and the U12 rows live in the chunk regions (points'
// powers, monomials, operands), which hold nothing during the solve.
void plan_lu_block(LdsPlan& L, int n) {
  L.lu_nb = 0;
  if (L.A_in_lds || n != 3) return;
  const long long free_dbl = (long long)L.off_fg - L.off_pow;
  for (int nb = 32; nb >= 4; nb -= 4)
    if (lu_ws_doubles(L.S, nb) <= free_dbl) {
      L.lu_nb = nb;
      return;
    }
}

int plan_lds(tdg_ctx* X, int forced_pch = 0) {
  const int n = X->topo.n;
  const Table& Tm = X->tabs[X->opts.p_max];
  LdsPlan& L = X->lp;
  int maxpatch = 0;
  for (int v = 0; v < X->topo.nv; ++v) maxpatch = std::max(maxpatch, X->topo.v2e_ptr[v + 1] - X->topo.v2e_ptr[v]);
  // recover_U = 2: the constant of every speed group joins the unknowns
  L.S = X->max_groups * (Tm.NW + (X->opts.recover_U == 2 ? 1 : 0));
  L.lda = L.S + 1 + ((L.S + 1) % 2 == 0 ? 1 : 0);
  const int ntd = (Tm.NW + 15) / 16;
  L.NWP = ntd * 16 + 1;
  const int ntiles = ntd * (ntd + 1) / 2;
  int tpw = (ntiles + kBlock / 64 - 1) / (kBlock / 64);
  L.TPW = 1;
  while (L.TPW < tpw) L.TPW *= 2;
  if (L.TPW > 16) L.TPW = 16;  // more tiles: several passes over the points
  L.M = Tm.M;
  L.maxpatch = maxpatch;
  L.ELS = el_size(n);
  L.maxfaces = 0;
  for (int v = 0; v < X->topo.nv; ++v) L.maxfaces = std::max(L.maxfaces, X->topo.vb_ptr[v + 1] - X->topo.vb_ptr[v]);
  if (L.maxfaces > kMaxFaces) return fail(TDG_EINVAL, "too many boundary facets at one vertex");
  const int nue = Tm.ue_ptr.back(), ntr = (int)Tm.tr_j.size();
  const int nint = (Tm.NW + 1) + nue * (n + 2) + ((n + 2) * Tm.M + 1) + ntr + Tm.M * (n + 1);
  L.tab_int_dbl = (nint + 1) / 2;
  const int tab_dbl = L.tab_int_dbl + nue * (n + 2) + ntr;
  struct Choice {
    bool a, t;
    int min_pch;
  };
  const Choice order[4] = {{true, true, 16}, {true, false, 16}, {false, true, 4}, {false, false, 4}};
  const int pmax = X->opts.p_max;
  for (int p = 0; p <= kMaxP; ++p) L.nwp[p] = p >= 1 && p <= pmax ? ((X->tabs[p].NW + 15) / 16) * 16 + 1 : 0;
  L.moment = (X->gram_mode == 1 && X->opts.precision == 0) ? 1 : 0;
  if (L.moment && X->opts.recover_U == 2)
    return fail(TDG_EINVAL, "the moment Gram does not form the recovery terms of recover_U = 2");
  if (L.moment) {
    // moment mode: W1 holds the moments and the bottom data moments (the Z row of
    // the Gram reuses the latter), later the write-back coefficients with the
    // monomial table, or the interface face values
    long long mom = 0;
    for (int p = 1; p <= pmax; ++p) {
      const Table& tb = X->tabs[p];
      mom = std::max(mom, (long long)(n + 1) * tb.M2 + (long long)(n + 1) * tb.M1 + tb.M);
      mom = std::max(mom, (((long long)(n + 2) * tb.M + 3) & ~3LL) + ((long long)tb.ntask1 * kTaskInts + 1) / 2);
    }
    for (int p = 1; p <= pmax; ++p) {
      // the per-face path (speed interfaces, Neumann faces) needs at least one
      // point per chunk: 4 face-value rows and the point's monomials
      mom = std::max(mom, 4LL * (((X->tabs[p].NW + 15) / 16) * 16 + 1) + X->tabs[p].M1);
      // the matrix-core evaluation of the 3+1D write-back
      if (n == 3 && X->tabs[p].ev_nl) mom = std::max(mom, ev_doubles(p, X->tabs[p].ev_nl));
    }
    for (int p = 1; p <= pmax; ++p)
      if (X->tabs[p].ntask2 > kTaskSlots * kBlock || X->tabs[p].ntask1 > kTaskSlots1 * kBlock)
        return fail(TDG_EINVAL, "too many moment tasks for the moment mode at this degree");
    for (const Choice& ch : order) {
      for (int pch : {64, 32, 16, 8, 4}) {
        if (forced_pch ? pch != forced_pch : pch < ch.min_pch) continue;
        L.PCH = pch;
        L.A_in_lds = ch.a;
        L.tab_in_lds = ch.t;
        // (sections 5 and 6 evaluate one point per thread: no monomial table)
        const long long w1 = mom;
        long long pw_sz = 0;
        for (int p = 1; p <= pmax; ++p) {
          L.pch[p] = pch;
          int c = pch;
          while (c > 1 && 4LL * c * L.nwp[p] + (long long)X->tabs[p].M1 * c > w1) c /= 2;
          L.pci[p] = c;
          pw_sz = std::max(pw_sz, std::max((long long)pch * (n + 1) * (3 * p), 2LL * pch * (n + 1) * (p + 1)));
        }
        int off = 0;
        auto take = [&](long long cnt) {
          int o = off;
          off += (int)((cnt + 3) & ~3LL);
          return o;
        };
        L.off_x = take(L.S + kMaxGroups);
        L.off_el = take((long long)maxpatch * L.ELS);
        L.off_misc = take(5 * kMaxGroups + 24 + (long long)X->max_groups * L.NWP);
        L.off_pt = take((long long)pch * (2 * (n + 1) + 1 + (n + 2) + n + 1));
        L.off_pow = take(pw_sz);
        L.off_mono = 0;
        L.off_W1 = take(w1);
        L.off_fg = take((long long)std::max(L.maxfaces, 1) * (2 + n + (n + 1) * (n + 1)));
        L.off_tab = ch.t ? take(tab_dbl) : 0;
        L.off_A = ch.a ? take((long long)L.S * L.lda) : 0;
        L.off_AF = 0;
        L.off_vec = 0;
        L.total = off;
        if ((size_t)L.total * sizeof(double) + 1024 <= 160 * 1024) {
          plan_lu_block(L, n);
          // lower degrees: a larger moment chunk in the free tail of W1
          const long long w1_have = (long long)L.off_fg - L.off_W1;
          for (int p = 0; p <= kMaxP; ++p) {
            L.mpch[p] = L.pch[p];
            L.moff[p] = -1;
          }
          if (n == 3)
            for (int p = 2; p <= pmax; ++p) {
              const Table& tb = X->tabs[p];
              if (!tb.mt_ntile) continue;
              const long long used = ((long long)(n + 1) * tb.M2 + (long long)(n + 1) * tb.M1 + tb.M + 3) & ~3LL;
              for (int cand : {64, 32}) {
                if (cand <= L.pch[p]) break;
                const long long need = (long long)cand * (2 * (n + 1) + 1 + (n + 2)) +
                                       (long long)cand * (n + 1) * ((2 * p - 1) + (p + 1));
                if (used + need <= w1_have) {
                  L.mpch[p] = cand;
                  L.moff[p] = (int)used;
                  break;
                }
              }
            }
          return TDG_OK;
        }
      }
    }
    return fail(TDG_EINVAL, "tent kernel working set (moment mode) does not fit in LDS");
  }
  // per-point sizes (doubles) of the chunk regions at degree p with operand stride nwp
  auto pow_sz = [&](int p, long long c) { return 2LL * c * (n + 1) * (p + 1); };
  auto mono_sz = [&](int p, long long c) { return (long long)X->tabs[p].M * 2 * c; };
  // W1 also holds the write-back coefficients and the degree-p monomial runs
  // (the matrix-core evaluation of 3+1D write-backs runs where W1 happens to be
  // large enough for it, see solve_tent; it does not enlarge this plan)
  auto wb_sz = [&](int p) {
    return (((long long)(n + 2) * X->tabs[p].M + 3) & ~3LL) + ((long long)X->tabs[p].ntask1 * kTaskInts + 1) / 2;
  };
  auto w1_sz = [&](int p, long long c) {
    const long long nwp = ((X->tabs[p].NW + 15) / 16) * 16 + 1;
    return std::max<long long>(c * (n + 3) * nwp, wb_sz(p));
  };
  const long long pt_per = 2 * (n + 1) + 1 + (n + 2) + n + 1;
  for (int p = 0; p <= kMaxP; ++p) L.pch[p] = 0;
  for (const Choice& ch : order) {
    for (int pch : {64, 32, 16, 8, 4}) {
      if (forced_pch ? pch != forced_pch : pch < ch.min_pch) continue;
      L.PCH = pch;
      L.A_in_lds = ch.a;
      L.tab_in_lds = ch.t;
      // a lower degree takes the largest chunk whose monomial and operand regions
      // fit in the ones sized for p_max; the small point and power regions grow
      // with it while the whole plan fits (else lower degrees shrink back)
      for (int p = 1; p <= pmax; ++p) {
        int c = pch;
        if (p < pmax)
          for (int cand : {64, 32, 16, 8, 4})
            if (cand >= pch && mono_sz(p, cand) <= mono_sz(pmax, pch) && w1_sz(p, cand) <= w1_sz(pmax, pch)) {
              c = cand;
              break;
            }
        L.pch[p] = c;
      }
      for (;;) {
        for (int p = 1; p <= pmax; ++p) L.pci[p] = L.pch[p];
        long long pt_sz = 0, pw_sz = 0;
        for (int p = 1; p <= pmax; ++p) {
          pt_sz = std::max(pt_sz, L.pch[p] * pt_per);
          pw_sz = std::max(pw_sz, pow_sz(p, L.pch[p]));
        }
        int off = 0;
        auto take = [&](long long cnt) {
          int o = off;
          off += (int)((cnt + 3) & ~3LL);
          return o;
        };
        L.off_x = take(L.S + kMaxGroups);
        L.off_el = take((long long)maxpatch * L.ELS);
        L.off_misc = take(5 * kMaxGroups + 24 + (long long)X->max_groups * L.NWP);
        L.off_pt = take(pt_sz);
        L.off_pow = take(pw_sz);
        L.off_mono = take(mono_sz(pmax, pch));
        L.off_W1 = take(w1_sz(pmax, pch));
        L.off_fg = take((long long)std::max(L.maxfaces, 1) * (2 + n + (n + 1) * (n + 1)));
        L.off_tab = ch.t ? take(tab_dbl) : 0;
        L.off_A = ch.a ? take((long long)L.S * L.lda) : 0;
        const bool mixed = X->opts.precision == 1;
        L.off_AF = (mixed && ch.a) ? take((long long)L.S * L.lda) : 0;
        L.off_vec = mixed ? take(2LL * L.S) : 0;
        L.total = off;
        if ((size_t)L.total * sizeof(double) + 1024 <= 160 * 1024) {
          plan_lu_block(L, n);
          for (int p = 0; p <= kMaxP; ++p) {
            L.mpch[p] = L.pch[p];
            L.moff[p] = -1;
          }
          return TDG_OK;
        }
        // shrink the largest lower-degree chunk, if any is above the p_max chunk
        int pbig = 0;
        for (int p = 1; p < pmax; ++p)
          if (L.pch[p] > pch && (pbig == 0 || L.pch[p] > L.pch[pbig])) pbig = p;
        if (!pbig) break;
        L.pch[pbig] /= 2;
      }
    }
  }
  return fail(TDG_EINVAL, "tent kernel working set does not fit in LDS");
}

// Copies the per-degree descriptors (tables and the current plan) to the device.
int upload_tabd(tdg_ctx* X, hipStream_t stream, bool async) {
  for (int p = 1; p <= X->opts.p_max; ++p) {
    X->tabd[p].pch = X->lp.pch[p];
    X->tabd[p].nwp = X->lp.nwp[p];
    X->tabd[p].pci = X->lp.pci[p];
    X->tabd[p].mpch = X->lp.mpch[p];
    X->tabd[p].moff = X->lp.moff[p];
  }
  void* dst = (double*)X->dev[TDG_BUF_F64] + X->o_tabd;
  const size_t bytes = sizeof(TableDesc) * (kMaxP + 1);
  if (async) {
    if (hipMemcpyAsync(dst, X->tabd, bytes, hipMemcpyHostToDevice, stream) != hipSuccess) return -1;
    return hipStreamSynchronize(stream) == hipSuccess ? 0 : -1;
  }
  return hipMemcpy(dst, X->tabd, bytes, hipMemcpyHostToDevice) == hipSuccess ? 0 : -1;
}

}  // namespace

extern "C" {

const char* tdg_last_error(void) { return last_error_cstr(); }

int tent_pitch(const tdg_mesh* mesh, const double* c, double T, double gamma, tdg_tents** out) {
  TDG_TRY_BEGIN
  if (!mesh || !out) return fail(TDG_EINVAL, "NULL argument");
  *out = nullptr;
  Topology topo;
  std::string err;
  int rc = build_topology(*mesh, c, topo, err);
  if (rc) return fail(rc, err);
  auto* t = new tdg_tents();
  rc = pitch_tents(topo, T, gamma, t->list, err);
  if (rc) {
    delete t;
    return fail(rc, err);
  }
  *out = t;
  return TDG_OK;
  TDG_TRY_END
}

int tent_info(const tdg_tents* t, int32_t* n_layers, int64_t* n_tents, double* max_face_slope) {
  if (!t) return fail(TDG_EINVAL, "NULL tents");
  if (n_layers) *n_layers = (int32_t)t->list.layer_ptr.size() - 1;
  if (n_tents) *n_tents = (int64_t)t->list.V.size();
  if (max_face_slope) *max_face_slope = t->list.max_slope;
  return TDG_OK;
}

int tent_export(const tdg_tents* t, int32_t* vertex, double* t_bot, double* t_top, int64_t* layer_ptr) {
  if (!t) return fail(TDG_EINVAL, "NULL tents");
  const auto& L = t->list;
  if (vertex) std::copy(L.V.begin(), L.V.end(), vertex);
  if (t_bot) std::copy(L.tb.begin(), L.tb.end(), t_bot);
  if (t_top) std::copy(L.tt.begin(), L.tt.end(), t_top);
  if (layer_ptr) std::copy(L.layer_ptr.begin(), L.layer_ptr.end(), layer_ptr);
  return TDG_OK;
}

void tent_free(tdg_tents* t) { delete t; }

int trefftz_create(const tdg_mesh* mesh, const double* c, const tdg_tents* tents, const tdg_opts* opts,
                   tdg_ctx** out) {
  TDG_TRY_BEGIN
  if (!mesh || !tents || !opts || !out) return fail(TDG_EINVAL, "NULL argument");
  *out = nullptr;
  if (opts->p_max < 1 || opts->p_max > kMaxP) return fail(TDG_EINVAL, "p_max must be in 1..10");
  if (opts->q < 0 || opts->q > 16) return fail(TDG_EINVAL, "q must be in 0..16");
  if (opts->layout != 1) return fail(TDG_EINVAL, "layout must be 1 (values at quadrature points)");
  if (opts->precision != 0 && opts->precision != 1) return fail(TDG_EINVAL, "precision must be 0 or 1");
  if (!(opts->alpha > 0) || !(opts->beta > 0)) return fail(TDG_EINVAL, "alpha and beta must be positive");
  if (opts->recover_U < 0 || opts->recover_U > 2) return fail(TDG_EINVAL, "recover_U must be 0, 1 or 2");
  if (opts->seed_basis < 0 || opts->seed_basis > 2)
    return fail(TDG_EINVAL, "seed_basis must be 0 (monomials), 1 (Legendre) or 2 (Chebyshev)");
  if (opts->recover_U == 2 && opts->precision != 0)
    return fail(TDG_EINVAL, "recover_U = 2 (the recovery terms for every test function) needs precision = 0");
  auto X = new tdg_ctx();
  std::unique_ptr<tdg_ctx> guard(X);
  std::string err;
  int rc = build_topology(*mesh, c, X->topo, err);
  if (rc) return fail(rc, err);
  if (tents->list.n != mesh->dim) return fail(TDG_EINVAL, "tents were pitched on a mesh of another dimension");
  X->tents = tents->list;
  for (int v : X->tents.V)
    if (v < 0 || v >= X->topo.nv) return fail(TDG_EINVAL, "tent vertex out of range");
  X->opts = *opts;
  const int n = X->topo.n;
  const int q = opts->q ? opts->q : opts->p_max;
  X->quad = simplex_rule(n, q);
  X->tabs.resize(opts->p_max + 1);
  for (int p = 1; p <= opts->p_max; ++p) X->tabs[p] = build_table(n, p, opts->seed_basis);
  X->nq = (int64_t)X->topo.ne * X->quad.Q;
  // speed groups per patch
  for (int v = 0; v < X->topo.nv; ++v) {
    std::vector<double> cs;
    for (int i = X->topo.v2e_ptr[v]; i < X->topo.v2e_ptr[v + 1]; ++i) {
      double ce = X->topo.c[X->topo.v2e[i]];
      if (std::find(cs.begin(), cs.end(), ce) == cs.end()) cs.push_back(ce);
    }
    X->max_groups = std::max(X->max_groups, (int)cs.size());
  }
  if (X->max_groups > kMaxGroups) return fail(TDG_EINVAL, "more than 32 wave speeds in one vertex patch");
  // boundary points: replay the front
  {
    const int Q = X->quad.Q;
    const auto& tp = X->tents;
    const int64_t nt = (int64_t)tp.V.size();
    X->bpt_off.assign(nt + 1, 0);
    std::vector<double> tau(X->topo.nv, 0.0);
    for (int64_t i = 0; i < nt; ++i) {
      const int V = tp.V[i];
      if (tau[V] != tp.tb[i]) return fail(TDG_EINVAL, "tent list does not follow the front");
      // the points of the tent's Dirichlet faces, then of its Neumann faces
      const int nfd = X->topo.vb_ptr[V + 1] - X->topo.vb_ptr[V];
      const int nf = nfd + X->topo.vn_ptr[V + 1] - X->topo.vn_ptr[V];
      X->bpt_off[i + 1] = X->bpt_off[i] + (int64_t)nf * Q;
      for (int f = 0; f < nf; ++f) {
        const bool neu = f >= nfd;
        const int* fl = neu ? &X->topo.vn[2 * (X->topo.vn_ptr[V] + f - nfd)] : &X->topo.vb[2 * (X->topo.vb_ptr[V] + f)];
        const int e = fl[0], k = fl[1];
        double P[4][4];
        for (int d = 0; d < n; ++d) P[0][d] = P[1][d] = X->topo.coords[(size_t)V * n + d];
        P[0][n] = tp.tb[i];
        P[1][n] = tp.tt[i];
        int cc = 2;
        for (int l = 0; l <= n; ++l) {
          int w = X->topo.elems[(size_t)e * (n + 1) + l];
          if (l == k || w == V) continue;
          for (int d = 0; d < n; ++d) P[cc][d] = X->topo.coords[(size_t)w * n + d];
          P[cc][n] = tau[w];
          ++cc;
        }
        for (int qq = 0; qq < Q; ++qq) {
          double y[4] = {0, 0, 0, 0};
          for (int l = 0; l <= n; ++l)
            for (int d = 0; d <= n; ++d) y[d] += X->quad.lam[(size_t)qq * (n + 1) + l] * P[l][d];
          X->bpts.insert(X->bpts.end(), y, y + n + 1);
          X->bkind.push_back(neu ? 1 : 0);
        }
      }
      tau[V] = tp.tt[i];
    }
    X->nb = X->bpt_off[nt];
  }
  // stage the static tables
  const Topology& T = X->topo;
  X->o_coords = push(X->hf64, T.coords.data(), T.coords.size());
  X->o_c = push(X->hf64, T.c.data(), T.c.size());
  X->o_grad = push(X->hf64, T.grad_lam.data(), T.grad_lam.size());
  X->o_det = push(X->hf64, T.absdet.data(), T.absdet.size());
  X->o_lam = push(X->hf64, X->quad.lam.data(), X->quad.lam.size());
  X->o_w = push(X->hf64, X->quad.w.data(), X->quad.w.size());
  X->o_tb = push(X->hf64, X->tents.tb.data(), X->tents.tb.size());
  X->o_tt = push(X->hf64, X->tents.tt.data(), X->tents.tt.size());
  {
    std::vector<double> tmp(X->bpt_off.size());
    std::memcpy(tmp.data(), X->bpt_off.data(), tmp.size() * sizeof(double));
    X->o_bpt = push(X->hf64, tmp.data(), tmp.size());
  }
  X->o_elems = push(X->hi32, T.elems.data(), T.elems.size());
  X->o_v2e_ptr = push(X->hi32, T.v2e_ptr.data(), T.v2e_ptr.size());
  X->o_v2e = push(X->hi32, T.v2e.data(), T.v2e.size());
  X->o_vb_ptr = push(X->hi32, T.vb_ptr.data(), T.vb_ptr.size());
  X->o_vb = push(X->hi32, T.vb.data(), T.vb.size());
  X->o_vn_ptr = push(X->hi32, T.vn_ptr.data(), T.vn_ptr.size());
  X->o_vn = push(X->hi32, T.vn.data(), T.vn.size());
  X->o_vi_ptr = push(X->hi32, T.vi_ptr.data(), T.vi_ptr.size());
  X->o_vi = push(X->hi32, T.vi.data(), T.vi.size());
  X->o_tentV = push(X->hi32, X->tents.V.data(), X->tents.V.size());
  for (int p = 1; p <= opts->p_max; ++p) {
    const Table& tb = X->tabs[p];
    auto& o = X->toff[p];
    o.parent = push(X->hi32, tb.parent.data(), tb.parent.size());
    o.var = push(X->hi32, tb.var.data(), tb.var.size());
    o.expo = push(X->hi32, tb.expo.data(), tb.expo.size());
    o.fo_ptr = push(X->hi32, tb.fo_ptr.data(), tb.fo_ptr.size());
    o.fo_idx = push(X->hi32, tb.fo_idx.data(), tb.fo_idx.size());
    o.u_ptr = push(X->hi32, tb.u_ptr.data(), tb.u_ptr.size());
    o.u_idx = push(X->hi32, tb.u_idx.data(), tb.u_idx.size());
    o.ue_ptr = push(X->hi32, tb.ue_ptr.data(), tb.ue_ptr.size());
    o.ue_idx = push(X->hi32, tb.ue_idx.data(), tb.ue_idx.size());
    o.tr_ptr = push(X->hi32, tb.tr_ptr.data(), tb.tr_ptr.size());
    o.tr_j = push(X->hi32, tb.tr_j.data(), tb.tr_j.size());
    o.expo2 = push(X->hi32, tb.expo2.data(), tb.expo2.size());
    o.K2 = push(X->hi32, tb.K2.data(), tb.K2.size());
    o.task2 = push(X->hi32, tb.task2.data(), tb.task2.size());
    o.task1 = push(X->hi32, tb.task1.data(), tb.task1.size());
    o.mt_ex = push(X->hi32, tb.mt_ex.data(), tb.mt_ex.size());
    o.mt_map = push(X->hi32, tb.mt_map.data(), tb.mt_map.size());
    o.ev_ab = push(X->hi32, tb.ev_ab.data(), tb.ev_ab.size());
    o.ev_ex = push(X->hi32, tb.ev_ex.data(), tb.ev_ex.size());
    o.ue_coef = push(X->hf64, tb.ue_coef.data(), tb.ue_coef.size());
    o.tr_coef = push(X->hf64, tb.tr_coef.data(), tb.tr_coef.size());
    o.fo_coef = push(X->hf64, tb.fo_coef.data(), tb.fo_coef.size());
    o.u_coef = push(X->hf64, tb.u_coef.data(), tb.u_coef.size());
    std::vector<float> f32(tb.fo_coef.begin(), tb.fo_coef.end());
    if (f32.size() % 2) f32.push_back(0.0f);
    std::vector<double> packed(f32.size() / 2);
    std::memcpy(packed.data(), f32.data(), f32.size() * sizeof(float));
    o.fo_coef32 = push(X->hf64, packed.data(), packed.size());
  }
  {
    const size_t nd = (sizeof(TableDesc) * (kMaxP + 1) + 7) / 8;
    std::vector<double> zeros(nd, 0.0);
    X->o_tabd = push(X->hf64, zeros.data(), zeros.size());
  }
  rc = plan_lds(X);
  if (rc) return rc;
  // global system slots are needed if the systems do not fit in LDS in either
  // Gram mode (the mode can be switched after binding)
  bool need_slots = !X->lp.A_in_lds;
  if (X->opts.precision == 0 && X->opts.recover_U != 2) {
    const LdsPlan keep = X->lp;
    X->gram_mode = 1;
    if (plan_lds(X) == TDG_OK && !X->lp.A_in_lds) need_slots = true;
    X->gram_mode = 0;
    X->lp = keep;
  }
  // buffer sizes
  const int64_t nst = X->nq * (n + 2);
  X->sizes[TDG_BUF_F64] = (int64_t)X->hf64.size() * 8;
  X->sizes[TDG_BUF_I32] = (int64_t)X->hi32.size() * 4;
  X->sizes[TDG_BUF_STATE] = nst * 8;
  X->sizes[TDG_BUF_STATE0] = nst * 8;
  X->sizes[TDG_BUF_TAU] = (int64_t)T.nv * 8;
  X->sizes[TDG_BUF_GD] = std::max<int64_t>(X->nb, 1) * 8;
  X->w_ex = 0;
  X->w_partial = (size_t)(X->nq * (n + 1) + 31) / 32 * 32;
  X->w_out = X->w_partial + 2 * X->nblocks_red + 32;
  X->w_status = X->w_out + 32;
  X->w_ctr = X->w_status + 32;
  X->w_order = X->w_ctr + ((X->tents.layer_ptr.size() + 1) / 2 + 31) / 32 * 32;
  X->w_sys = X->w_order + ((X->tents.V.size() + 1) / 2 + 31) / 32 * 32;
  {
    int64_t widest = 0;
    for (size_t l = 0; l + 1 < X->tents.layer_ptr.size(); ++l)
      widest = std::max<int64_t>(widest, X->tents.layer_ptr[l + 1] - X->tents.layer_ptr[l]);
    X->sys_stride = need_slots ? ((int64_t)X->lp.S * X->lp.lda * (X->opts.precision == 1 ? 2 : 1) + 31) / 32 * 32 : 0;
    X->sizes[TDG_BUF_WORK] = (int64_t)(X->w_sys + X->sys_stride * widest) * 8;
  }
  X->sizes[TDG_BUF_TENT] = std::max<int64_t>((int64_t)X->tents.V.size(), 1) * 16;
  guard.release();
  *out = X;
  return TDG_OK;
  TDG_TRY_END
}

int trefftz_quad_points(const tdg_ctx* X, int64_t* nq, double* xq, double* w) {
  if (!X || !nq) return fail(TDG_EINVAL, "NULL argument");
  *nq = X->nq;
  const int n = X->topo.n, Q = X->quad.Q;
  for (int e = 0; e < X->topo.ne; ++e) {
    const int* vs = &X->topo.elems[(size_t)e * (n + 1)];
    for (int q = 0; q < Q; ++q) {
      const double* lam = &X->quad.lam[(size_t)q * (n + 1)];
      if (xq)
        for (int d = 0; d < n; ++d) {
          double s = 0.0;
          for (int k = 0; k <= n; ++k) s += lam[k] * X->topo.coords[(size_t)vs[k] * n + d];
          xq[((size_t)e * Q + q) * n + d] = s;
        }
      if (w) w[(size_t)e * Q + q] = X->quad.w[q] * X->topo.absdet[e];
    }
  }
  return TDG_OK;
}

int trefftz_boundary_points(const tdg_ctx* X, int64_t* nb, double* xt) {
  if (!X || !nb) return fail(TDG_EINVAL, "NULL argument");
  *nb = X->nb;
  if (xt) std::copy(X->bpts.begin(), X->bpts.end(), xt);
  return TDG_OK;
}

int trefftz_boundary_kinds(const tdg_ctx* X, int8_t* kind) {
  if (!X || !kind) return fail(TDG_EINVAL, "NULL argument");
  std::copy(X->bkind.begin(), X->bkind.end(), kind);
  return TDG_OK;
}

int tdg_boundary_facets(const tdg_mesh* mesh, int64_t* nbf, int32_t* facets) {
  TDG_TRY_BEGIN
  if (!mesh || !nbf) return fail(TDG_EINVAL, "NULL argument");
  tdg_mesh m = *mesh;
  m.bface_kind = nullptr;
  std::vector<double> ones(std::max(mesh->ne, 0), 1.0);
  Topology T;
  std::string err;
  const int rc = build_topology(m, ones.data(), T, err);
  if (rc) return fail(rc, err);
  *nbf = (int64_t)T.bfacets.size();
  if (facets)
    for (size_t i = 0; i < T.bfacets.size(); ++i) {
      facets[2 * i] = T.bfacets[i].first;
      facets[2 * i + 1] = T.bfacets[i].second;
    }
  return TDG_OK;
  TDG_TRY_END
}

int trefftz_buffer_sizes(const tdg_ctx* X, int64_t sizes[TDG_NBUF]) {
  if (!X || !sizes) return fail(TDG_EINVAL, "NULL argument");
  for (int i = 0; i < TDG_NBUF; ++i) sizes[i] = X->sizes[i];
  return TDG_OK;
}

int trefftz_bind(tdg_ctx* X, void* const dev_ptrs[TDG_NBUF], tdg_stream stream) {
  if (!X || !dev_ptrs) return fail(TDG_EINVAL, "NULL argument");
  for (int i = 0; i < TDG_NBUF; ++i) {
    if (!dev_ptrs[i]) return fail(TDG_EINVAL, "NULL device buffer");
    if (((uintptr_t)dev_ptrs[i]) % 256) return fail(TDG_EINVAL, "device buffer not 256-byte aligned");
    X->dev[i] = dev_ptrs[i];
  }
  hipStream_t st = (hipStream_t)stream;
  HIP_OK(hipMemcpyAsync(X->dev[TDG_BUF_F64], X->hf64.data(), X->hf64.size() * 8, hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(X->dev[TDG_BUF_I32], X->hi32.data(), X->hi32.size() * 4, hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  const double* F = (const double*)X->dev[TDG_BUF_F64];
  const int* I = (const int*)X->dev[TDG_BUF_I32];
  KParams& P = X->kp;
  const Topology& T = X->topo;
  P.n = T.n;
  P.nv = T.nv;
  P.ne = T.ne;
  P.Q = X->quad.Q;
  P.pmax = X->opts.p_max;
  P.ntents = (int)X->tents.V.size();
  P.precision = X->opts.precision;
  P.recover_U = X->opts.recover_U;
  P.alpha = X->opts.alpha;
  P.beta = X->opts.beta;
  P.coords = F + X->o_coords;
  P.c = F + X->o_c;
  P.grad_lam = F + X->o_grad;
  P.absdet = F + X->o_det;
  P.lam_ref = F + X->o_lam;
  P.w_ref = F + X->o_w;
  P.tent_tb = F + X->o_tb;
  P.tent_tt = F + X->o_tt;
  P.bpt_off = (const long long*)(F + X->o_bpt);
  P.elems = I + X->o_elems;
  P.v2e_ptr = I + X->o_v2e_ptr;
  P.v2e = I + X->o_v2e;
  P.vb_ptr = I + X->o_vb_ptr;
  P.vb = I + X->o_vb;
  P.vn_ptr = I + X->o_vn_ptr;
  P.vn = I + X->o_vn;
  P.vi_ptr = I + X->o_vi_ptr;
  P.vi = I + X->o_vi;
  P.tent_V = I + X->o_tentV;
  P.p_per_tent = nullptr;
  P.state = (double*)X->dev[TDG_BUF_STATE];
  P.tau = (double*)X->dev[TDG_BUF_TAU];
  P.gD = (const double*)X->dev[TDG_BUF_GD];
  double* W = (double*)X->dev[TDG_BUF_WORK];
  P.status = (int*)(W + X->w_status);
  P.dissip = (double*)X->dev[TDG_BUF_TENT];
  P.ir_steps = (int*)((double*)X->dev[TDG_BUF_TENT] + X->tents.V.size());
  P.work = W + X->w_sys;
  P.work_stride = X->sys_stride;
  P.p_fixed = 0;
  P.indicator = 0;
  P.write_back = 1;
  P.eta_tol = 0.0;
  P.p_used = nullptr;
  for (int p = 0; p <= kMaxP; ++p) X->tabd[p] = TableDesc{};
  for (int p = 1; p <= X->opts.p_max; ++p) {
    const Table& tb = X->tabs[p];
    const auto& o = X->toff[p];
    TableDesc& D = X->tabd[p];
    D.p = p;
    D.NW = tb.NW;
    D.M = tb.M;
    D.M1 = tb.M1;
    D.M2 = tb.M2;
    D.expo2 = I + o.expo2;
    D.K2 = I + o.K2;
    D.task2 = I + o.task2;
    D.task1 = I + o.task1;
    D.ntask2 = tb.ntask2;
    D.ntask1 = tb.ntask1;
    D.mt_ntile = tb.mt_ntile;
    D.mt_ex = I + o.mt_ex;
    D.mt_map = I + o.mt_map;
    D.ev_nl = tb.ev_nl;
    D.ev_nat = tb.ev_nat;
    for (int i = 0; i < 8; ++i) D.ev_nks[i] = tb.ev_nks[i];
    for (int i = 0; i < 8; ++i) D.ev_nkv[i] = tb.ev_nkv[i];
    D.ev_ab = I + o.ev_ab;
    D.ev_ex = I + o.ev_ex;
    D.fo_nnz = (int)tb.fo_idx.size();
    D.u_nnz = (int)tb.u_idx.size();
    D.ue_n = tb.ue_ptr.back();
    D.tr_n = (int)tb.tr_j.size();
    D.ue_ptr = I + o.ue_ptr;
    D.ue_idx = I + o.ue_idx;
    D.ue_coef = F + o.ue_coef;
    D.tr_ptr = I + o.tr_ptr;
    D.tr_j = I + o.tr_j;
    D.tr_coef = F + o.tr_coef;
    D.parent = I + o.parent;
    D.var = I + o.var;
    D.expo = I + o.expo;
    D.fo_ptr = I + o.fo_ptr;
    D.fo_idx = I + o.fo_idx;
    D.fo_coef = F + o.fo_coef;
    D.fo_coef32 = (const float*)(F + o.fo_coef32);
    D.u_ptr = I + o.u_ptr;
    D.u_idx = I + o.u_idx;
    D.u_coef = F + o.u_coef;
  }
  P.tabd = (const TableDesc*)(F + X->o_tabd);
  if (upload_tabd(X, st, true)) return fail(TDG_EHIP, "upload of the degree descriptors failed");
  if (set_kernel_smem_limit(T.n, (size_t)X->lp.total * 8 + 64)) return fail(TDG_EHIP, "cannot raise the LDS limit");
  {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&X->ncu, hipDeviceAttributeMultiprocessorCount, dev));
    X->resident = resident_blocks_per_cu(T.n, X->lp.moment ? 0 : X->lp.TPW, X->opts.precision == 1, (size_t)X->lp.total * 8);
  }
  // clear state, front, status, per-tent outputs
  if (launch_fill(P.state, 0.0, X->nq * (T.n + 2), stream) || launch_fill(P.tau, 0.0, T.nv, stream) ||
      launch_fill(W + X->w_status, 0.0, 32, stream) ||
      launch_fill(P.dissip, 0.0, std::max<int64_t>((int64_t)X->tents.V.size(), 1) * 2, stream) ||
      launch_fill((double*)X->dev[TDG_BUF_GD], 0.0, std::max<int64_t>(X->nb, 1), stream))
    return fail(TDG_EHIP, "fill kernel launch failed");
  HIP_OK(hipStreamSynchronize(st));
  X->bound = true;
  return TDG_OK;
}

int trefftz_set_initial(tdg_ctx* X, const double* v0, const double* sigma0, const double* U0, tdg_stream stream) {
  TDG_TRY_BEGIN
  if (!X || !v0 || !sigma0) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  const int n = X->topo.n, Q = X->quad.Q, ne = X->topo.ne;
  std::vector<double> st((size_t)X->nq * (n + 2));
  for (int e = 0; e < ne; ++e)
    for (int q = 0; q < Q; ++q) {
      const size_t i = (size_t)e * Q + q;
      double* base = &st[(size_t)e * (n + 2) * Q];
      base[q] = v0[i];
      for (int d = 0; d < n; ++d) base[(size_t)(1 + d) * Q + q] = sigma0[i * n + d];
      base[(size_t)(n + 1) * Q + q] = U0 ? U0[i] : 0.0;
    }
  for (double x : st)
    if (!std::isfinite(x)) return fail(TDG_ENAN, "non-finite initial data");
  hipStream_t s = (hipStream_t)stream;
  HIP_OK(hipMemcpyAsync(X->dev[TDG_BUF_STATE0], st.data(), st.size() * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipStreamSynchronize(s));
  return trefftz_reset(X, stream);
  TDG_TRY_END
}

int trefftz_set_boundary(tdg_ctx* X, const double* gD, tdg_stream stream) {
  if (!X || (!gD && X->nb)) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  for (int64_t i = 0; i < X->nb; ++i)
    if (!std::isfinite(gD[i])) return fail(TDG_ENAN, "non-finite boundary data");
  hipStream_t s = (hipStream_t)stream;
  if (X->nb) HIP_OK(hipMemcpyAsync(X->dev[TDG_BUF_GD], gD, X->nb * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipStreamSynchronize(s));
  return TDG_OK;
}

int trefftz_reset(tdg_ctx* X, tdg_stream stream) {
  if (!X) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  hipStream_t s = (hipStream_t)stream;
  HIP_OK(hipMemcpyAsync(X->dev[TDG_BUF_STATE], X->dev[TDG_BUF_STATE0], X->sizes[TDG_BUF_STATE],
                        hipMemcpyDeviceToDevice, s));
  if (launch_fill(X->kp.tau, 0.0, X->topo.nv, stream) ||
      launch_fill(X->kp.dissip, 0.0, std::max<int64_t>((int64_t)X->tents.V.size(), 1) * 2, stream))
    return fail(TDG_EHIP, "fill kernel launch failed");
  return TDG_OK;
}

int trefftz_layer_solve(tdg_ctx* X, int32_t layer_begin, int32_t layer_end, const int8_t* p_per_tent,
                        tdg_stream stream) {
  if (!X) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  const int nl = (int)X->tents.layer_ptr.size() - 1;
  if (layer_begin < 0 || layer_end > nl || layer_begin > layer_end) return fail(TDG_EINVAL, "layer range out of bounds");
  KParams P = X->kp;
  P.p_per_tent = (const signed char*)p_per_tent;
  int* ctr = (int*)((double*)X->dev[TDG_BUF_WORK] + X->w_ctr);
  if (X->persistent && layer_end > layer_begin &&
      launch_fill((double*)X->dev[TDG_BUF_WORK] + X->w_ctr, 0.0, ((long long)nl + 1 + 1) / 2, stream))
    return fail(TDG_EHIP, "fill kernel launch failed");
  const int grid_max = std::max(1, X->ncu * X->resident);
  for (int l = layer_begin; l < layer_end; ++l) {
    const int t0 = (int)X->tents.layer_ptr[l];
    const int cnt = (int)(X->tents.layer_ptr[l + 1] - X->tents.layer_ptr[l]);
    const int g = std::min(cnt, grid_max);
    if (launch_layer(P, X->lp, t0, cnt, g, X->persistent ? ctr + l : nullptr, stream))
      return fail(TDG_EHIP, "tent kernel launch failed");
  }
  return TDG_OK;
}

int trefftz_set_indicator(tdg_ctx* X, int32_t on) {
  if (!X) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  X->kp.indicator = on ? 1 : 0;
  return TDG_OK;
}

int trefftz_tent_features(tdg_ctx* X, int32_t layer, float* feats, tdg_stream stream) {
  if (!X || !feats) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  const int nl = (int)X->tents.layer_ptr.size() - 1;
  if (layer < 0 || layer >= nl) return fail(TDG_EINVAL, "layer out of bounds");
  const int t0 = (int)X->tents.layer_ptr[layer];
  const int cnt = (int)(X->tents.layer_ptr[layer + 1] - t0);
  if (launch_features(X->kp, t0, cnt, feats, stream)) return fail(TDG_EHIP, "feature kernel launch failed");
  return TDG_OK;
}

int trefftz_layer_indicator(tdg_ctx* X, int32_t layer, int32_t p, double* eta, tdg_stream stream) {
  if (!X || !eta) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  const int nl = (int)X->tents.layer_ptr.size() - 1;
  if (layer < 0 || layer >= nl) return fail(TDG_EINVAL, "layer out of bounds");
  if (p < 1 || p > X->opts.p_max) return fail(TDG_EINVAL, "degree outside [1, p_max]");
  KParams P = X->kp;
  P.p_per_tent = nullptr;
  P.p_fixed = p;
  P.indicator = 1;
  P.write_back = 0;
  P.eta_tol = 0.0;
  P.dissip = eta;
  P.p_used = nullptr;
  const int t0 = (int)X->tents.layer_ptr[layer];
  const int cnt = (int)(X->tents.layer_ptr[layer + 1] - t0);
  const int g = std::min(cnt, std::max(1, X->ncu * X->resident));
  int* ctr = (int*)((double*)X->dev[TDG_BUF_WORK] + X->w_ctr);
  if (X->persistent && cnt > 0 && launch_fill((double*)X->dev[TDG_BUF_WORK] + X->w_ctr + layer / 2, 0.0, 1, stream))
    return fail(TDG_EHIP, "fill kernel launch failed");
  if (launch_layer(P, X->lp, t0, cnt, g, X->persistent ? ctr + layer : nullptr, stream))
    return fail(TDG_EHIP, "tent kernel launch failed");
  return TDG_OK;
}

int trefftz_layer_solve_adaptive(tdg_ctx* X, int32_t layer_begin, int32_t layer_end, const uint16_t* w_bf16,
                                 float log_eta_tol, double eta_tol, float* feats, int8_t* p_sel, int8_t* p_used,
                                 double* eta, tdg_stream stream) {
  if (!X || !feats || !p_sel) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  const int nl = (int)X->tents.layer_ptr.size() - 1;
  if (layer_begin < 0 || layer_end > nl || layer_begin > layer_end) return fail(TDG_EINVAL, "layer range out of bounds");
  if (!(eta_tol >= 0.0)) return fail(TDG_EINVAL, "eta_tol must be >= 0");
  KParams P = X->kp;
  P.p_per_tent = (const signed char*)p_sel;
  P.eta_tol = w_bf16 ? eta_tol : 0.0;
  P.p_used = (signed char*)p_used;
  if (eta) {
    P.dissip = eta;
    P.indicator = 1;
  }
  int* ctr = (int*)((double*)X->dev[TDG_BUF_WORK] + X->w_ctr);
  if (X->persistent && layer_end > layer_begin &&
      launch_fill((double*)X->dev[TDG_BUF_WORK] + X->w_ctr, 0.0, ((long long)nl + 1 + 1) / 2, stream))
    return fail(TDG_EHIP, "fill kernel launch failed");
  const int grid_max = std::max(1, X->ncu * X->resident);
  for (int l = layer_begin; l < layer_end; ++l) {
    const int t0 = (int)X->tents.layer_ptr[l];
    const int cnt = (int)(X->tents.layer_ptr[l + 1] - X->tents.layer_ptr[l]);
    P.order = nullptr;
    if (w_bf16) {
      // the chosen degrees, then the layer's queue in decreasing degree
      int* order = (int*)((double*)X->dev[TDG_BUF_WORK] + X->w_order);
      if (launch_features(P, t0, cnt, feats, stream) ||
          launch_select((const unsigned short*)w_bf16, feats, t0, cnt, log_eta_tol, X->opts.p_max,
                        (signed char*)p_sel, stream) ||
          launch_order((const signed char*)p_sel, t0, cnt, X->opts.p_max, order, stream))
        return fail(TDG_EHIP, "degree selection launch failed");
      P.order = order;
    } else if (launch_fill_i8((signed char*)p_sel + t0, (signed char)X->opts.p_max, cnt, stream)) {
      return fail(TDG_EHIP, "fill kernel launch failed");
    }
    if (launch_layer(P, X->lp, t0, cnt, std::min(cnt, grid_max), X->persistent ? ctr + l : nullptr, stream))
      return fail(TDG_EHIP, "tent kernel launch failed");
  }
  return TDG_OK;
}

static int read_status(tdg_ctx* X, hipStream_t s) {
  int st = 0;
  HIP_OK(hipMemcpyAsync(&st, (double*)X->dev[TDG_BUF_WORK] + X->w_status, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (st & kStatSingular) return fail(TDG_ESINGULAR, "a local tent system had a zero pivot");
  if (st & kStatNan) return fail(TDG_ENAN, "non-finite values in a tent solution");
  if (st & kStatNoConv) return fail(TDG_ENOCONV, "mixed-precision refinement did not converge");
  if (st & (kStatPatch | kStatGroups | kStatSize))
    return fail(TDG_EINVAL, "a tent exceeded the kernel's size limits (patch, groups or degree)");
  return TDG_OK;
}

int trefftz_status(tdg_ctx* X, tdg_stream stream) {
  if (!X || !X->bound) return fail(TDG_ESTATE, "context not bound");
  return read_status(X, (hipStream_t)stream);
}

int trefftz_eval_error(tdg_ctx* X, const double* v_ex, const double* sigma_ex, double* e_abs, double* e_rel,
                       tdg_stream stream) {
  if (!X || !v_ex || !sigma_ex) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  hipStream_t s = (hipStream_t)stream;
  double* W = (double*)X->dev[TDG_BUF_WORK];
  const int n = X->topo.n;
  HIP_OK(hipMemcpyAsync(W + X->w_ex, v_ex, X->nq * 8, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemcpyAsync(W + X->w_ex + X->nq, sigma_ex, X->nq * n * 8, hipMemcpyHostToDevice, s));
  if (launch_norms(X->kp, 0, W + X->w_ex, W + X->w_partial, X->nblocks_red, W + X->w_out, stream))
    return fail(TDG_EHIP, "reduction launch failed");
  double out[2];
  HIP_OK(hipMemcpyAsync(out, W + X->w_out, 16, hipMemcpyDeviceToHost, s));
  int rc = read_status(X, s);
  if (rc) return rc;
  const double ea = std::sqrt(out[0]);
  if (e_abs) *e_abs = ea;
  if (e_rel) *e_rel = out[1] > 0 ? ea / std::sqrt(out[1]) : INFINITY;
  return std::isfinite(ea) ? TDG_OK : fail(TDG_ENAN, "non-finite error");
}

int trefftz_eval_u_error(tdg_ctx* X, const double* U_ex, double* e_abs, double* e_rel, tdg_stream stream) {
  if (!X || !U_ex) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  hipStream_t s = (hipStream_t)stream;
  double* W = (double*)X->dev[TDG_BUF_WORK];
  HIP_OK(hipMemcpyAsync(W + X->w_ex, U_ex, X->nq * 8, hipMemcpyHostToDevice, s));
  if (launch_norms(X->kp, 2, W + X->w_ex, W + X->w_partial, X->nblocks_red, W + X->w_out, stream))
    return fail(TDG_EHIP, "reduction launch failed");
  double out[2];
  HIP_OK(hipMemcpyAsync(out, W + X->w_out, 16, hipMemcpyDeviceToHost, s));
  int rc = read_status(X, s);
  if (rc) return rc;
  const double ea = std::sqrt(out[0]);
  if (e_abs) *e_abs = ea;
  if (e_rel) *e_rel = out[1] > 0 ? ea / std::sqrt(out[1]) : INFINITY;
  return std::isfinite(ea) ? TDG_OK : fail(TDG_ENAN, "non-finite error");
}

int trefftz_energy(tdg_ctx* X, double* E_front, double* dissipated, tdg_stream stream) {
  if (!X) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  hipStream_t s = (hipStream_t)stream;
  double* W = (double*)X->dev[TDG_BUF_WORK];
  if (launch_norms(X->kp, 1, nullptr, W + X->w_partial, X->nblocks_red, W + X->w_out, stream))
    return fail(TDG_EHIP, "reduction launch failed");
  double out[2];
  HIP_OK(hipMemcpyAsync(out, W + X->w_out, 16, hipMemcpyDeviceToHost, s));
  std::vector<double> dis(X->tents.V.size());
  if (!dis.empty())
    HIP_OK(hipMemcpyAsync(dis.data(), X->kp.dissip, dis.size() * 8, hipMemcpyDeviceToHost, s));
  int rc = read_status(X, s);
  if (rc) return rc;
  if (E_front) *E_front = out[0];
  if (dissipated) {
    double sum = 0.0;
    for (double d : dis) sum += d;
    *dissipated = sum;
  }
  return TDG_OK;
}

int trefftz_read_state(tdg_ctx* X, double* v, double* sigma, double* U, tdg_stream stream) {
  TDG_TRY_BEGIN
  if (!X) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  const int n = X->topo.n, Q = X->quad.Q, ne = X->topo.ne;
  std::vector<double> st((size_t)X->nq * (n + 2));
  hipStream_t s = (hipStream_t)stream;
  HIP_OK(hipMemcpyAsync(st.data(), X->dev[TDG_BUF_STATE], st.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  for (int e = 0; e < ne; ++e)
    for (int q = 0; q < Q; ++q) {
      const size_t i = (size_t)e * Q + q;
      const double* base = &st[(size_t)e * (n + 2) * Q];
      if (v) v[i] = base[q];
      if (sigma)
        for (int d = 0; d < n; ++d) sigma[i * n + d] = base[(size_t)(1 + d) * Q + q];
      if (U) U[i] = base[(size_t)(n + 1) * Q + q];
    }
  return TDG_OK;
  TDG_TRY_END
}

int trefftz_table_info(const tdg_ctx* X, int32_t p, int32_t* N, int32_t* nnz_fields, int32_t* n_mono, int32_t* Q) {
  if (!X) return fail(TDG_EINVAL, "NULL argument");
  if (p < 1 || p > X->opts.p_max) return fail(TDG_EINVAL, "p out of range");
  const Table& t = X->tabs[p];
  if (N) *N = t.NW + 1;
  if (nnz_fields) *nnz_fields = (int32_t)t.fo_idx.size();
  if (n_mono) *n_mono = t.M;
  if (Q) *Q = X->quad.Q;
  return TDG_OK;
}

static void drop_graph(tdg_ctx* X) {
  if (X->graph_exec) hipGraphExecDestroy(X->graph_exec);
  if (X->graph) hipGraphDestroy(X->graph);
  X->graph_exec = nullptr;
  X->graph = nullptr;
}

int trefftz_set_tuning(tdg_ctx* X, int32_t pts_per_chunk, int32_t persistent) {
  if (!X) return fail(TDG_EINVAL, "NULL argument");
  if (persistent != 0 && persistent != 1) return fail(TDG_EINVAL, "persistent must be 0 or 1");
  if (pts_per_chunk != 0 && pts_per_chunk != 4 && pts_per_chunk != 8 && pts_per_chunk != 16 && pts_per_chunk != 32 &&
      pts_per_chunk != 64)
    return fail(TDG_EINVAL, "pts_per_chunk must be 0, 4, 8, 16, 32 or 64");
  const LdsPlan old = X->lp;
  int rc = plan_lds(X, pts_per_chunk);
  if (rc == TDG_OK && !X->lp.A_in_lds && X->sys_stride == 0)
    rc = fail(TDG_EINVAL, "shape puts the systems in global slots that were not allocated");
  if (rc != TDG_OK) {
    X->lp = old;
    return rc;
  }
  X->forced_pch = pts_per_chunk;
  X->persistent = persistent;
  // a captured sweep holds the old plan (LDS carve-up, kernel) in its kernel
  // nodes while the descriptors in device memory follow the new one: drop it
  drop_graph(X);
  if (X->bound) {
    if (upload_tabd(X, nullptr, false)) return fail(TDG_EHIP, "upload of the degree descriptors failed");
    if (set_kernel_smem_limit(X->topo.n, (size_t)X->lp.total * 8 + 64)) return fail(TDG_EHIP, "cannot raise the LDS limit");
    X->resident = resident_blocks_per_cu(X->topo.n, X->lp.moment ? 0 : X->lp.TPW, X->opts.precision == 1, (size_t)X->lp.total * 8);
  }
  return TDG_OK;
}

int trefftz_set_gram_mode(tdg_ctx* X, int32_t mode) {
  if (!X) return fail(TDG_EINVAL, "NULL argument");
  if (mode != 0 && mode != 1) return fail(TDG_EINVAL, "mode must be 0 or 1");
  if (mode == 1 && X->opts.precision != 0) return fail(TDG_EINVAL, "the moment Gram is FP64 only");
  const LdsPlan old = X->lp;
  const int old_mode = X->gram_mode;
  X->gram_mode = mode;
  int rc = plan_lds(X, X->forced_pch);
  if (rc == TDG_OK && !X->lp.A_in_lds && X->sys_stride == 0)
    rc = fail(TDG_EINVAL, "mode puts the systems in global slots that were not allocated");
  if (rc != TDG_OK) {
    X->lp = old;
    X->gram_mode = old_mode;
    return rc;
  }
  drop_graph(X);  // (see trefftz_set_tuning)
  if (X->bound) {
    if (upload_tabd(X, nullptr, false)) return fail(TDG_EHIP, "upload of the degree descriptors failed");
    if (set_kernel_smem_limit(X->topo.n, (size_t)X->lp.total * 8 + 64)) return fail(TDG_EHIP, "cannot raise the LDS limit");
    X->resident = resident_blocks_per_cu(X->topo.n, X->lp.moment ? 0 : X->lp.TPW, X->opts.precision == 1, (size_t)X->lp.total * 8);
  }
  return TDG_OK;
}

int trefftz_get_gram_mode(const tdg_ctx* X, int32_t* mode) {
  if (!X || !mode) return fail(TDG_EINVAL, "NULL argument");
  *mode = X->gram_mode;
  return TDG_OK;
}

int trefftz_get_tuning(const tdg_ctx* X, int32_t* pts_per_chunk, int32_t* persistent, int32_t* lds_bytes) {
  if (!X) return fail(TDG_EINVAL, "NULL argument");
  if (pts_per_chunk) *pts_per_chunk = X->lp.PCH;
  if (persistent) *persistent = X->persistent;
  if (lds_bytes) *lds_bytes = X->lp.total * 8;
  return TDG_OK;
}

int trefftz_capture_sweep(tdg_ctx* X, int32_t layer_begin, int32_t layer_end, const int8_t* p_per_tent,
                          int32_t with_reset, tdg_stream stream) {
  if (!X) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  if (!stream) return fail(TDG_EINVAL, "capture needs a non-default stream");
  drop_graph(X);
  hipStream_t s = (hipStream_t)stream;
  HIP_OK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = with_reset ? trefftz_reset(X, stream) : TDG_OK;
  if (rc == TDG_OK) rc = trefftz_layer_solve(X, layer_begin, layer_end, p_per_tent, stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (rc != TDG_OK) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(TDG_EHIP, std::string("stream capture failed: ") + hipGetErrorString(e));
  X->graph = g;
  e = hipGraphInstantiate(&X->graph_exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(X);
    return fail(TDG_EHIP, std::string("graph instantiation failed: ") + hipGetErrorString(e));
  }
  return TDG_OK;
}

int trefftz_replay_sweep(tdg_ctx* X, tdg_stream stream) {
  if (!X) return fail(TDG_EINVAL, "NULL argument");
  if (!X->graph_exec) return fail(TDG_ESTATE, "trefftz_capture_sweep first");
  HIP_OK(hipGraphLaunch(X->graph_exec, (hipStream_t)stream));
  return TDG_OK;
}

int trefftz_tent_stats(tdg_ctx* X, int64_t first_tent, int64_t count, int32_t* ir_steps, double* dissipation,
                       tdg_stream stream) {
  if (!X) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  const int64_t nt = (int64_t)X->tents.V.size();
  if (first_tent < 0 || count < 0 || first_tent + count > nt) return fail(TDG_EINVAL, "tent range out of bounds");
  hipStream_t s = (hipStream_t)stream;
  if (ir_steps && count)
    HIP_OK(hipMemcpyAsync(ir_steps, X->kp.ir_steps + first_tent, count * 4, hipMemcpyDeviceToHost, s));
  if (dissipation && count)
    HIP_OK(hipMemcpyAsync(dissipation, X->kp.dissip + first_tent, count * 8, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return TDG_OK;
}

// Internal (not part of include/tdg.h): the moment tables of degree p and the
// current LDS plan, host copies, for the host-side replay of the kernel's index
// arithmetic in the tests.  info[16] = {M, M1, M2, ntask2, ntask1, mt_ntile, Q,
// pch[p], off_pt, off_pow, off_W1, off_fg, total, moment, n, pmax}; each array
// (nullable) receives the table as built (task words, mt_ex, mt_map).
int tdg_debug_moment_tables(const tdg_ctx* X, int32_t p, int32_t* info, int32_t* task2, int32_t* task1,
                            int32_t* mt_ex, int32_t* mt_map) {
  if (!X || !info) return fail(TDG_EINVAL, "NULL argument");
  if (p < 1 || p > X->opts.p_max) return fail(TDG_EINVAL, "p out of range");
  const Table& t = X->tabs[p];
  const LdsPlan& L = X->lp;
  const int32_t v[16] = {t.M, t.M1, t.M2, t.ntask2, t.ntask1, t.mt_ntile, X->quad.Q, L.pch[p], L.off_pt,
                         L.off_pow, L.off_W1, L.off_fg, L.total, L.moment, X->topo.n, X->opts.p_max};
  std::copy(v, v + 16, info);
  if (task2) std::copy(t.task2.begin(), t.task2.end(), task2);
  if (task1) std::copy(t.task1.begin(), t.task1.end(), task1);
  if (mt_ex) std::copy(t.mt_ex.begin(), t.mt_ex.end(), mt_ex);
  if (mt_map) std::copy(t.mt_map.begin(), t.mt_map.end(), mt_map);
  return TDG_OK;
}

// Internal (tests): the queue order of layer `layer` as the last degree-adaptive
// solve left it (out: the layer's tent count of tent indices); synchronises.
int tdg_debug_queue_order(tdg_ctx* X, int32_t layer, int32_t* out, tdg_stream stream) {
  if (!X || !out) return fail(TDG_EINVAL, "NULL argument");
  if (!X->bound) return fail(TDG_ESTATE, "trefftz_bind first");
  const int nl = (int)X->tents.layer_ptr.size() - 1;
  if (layer < 0 || layer >= nl) return fail(TDG_EINVAL, "layer out of range");
  const int64_t t0 = X->tents.layer_ptr[layer], cnt = X->tents.layer_ptr[layer + 1] - t0;
  hipStream_t s = (hipStream_t)stream;
  const int* order = (const int*)((double*)X->dev[TDG_BUF_WORK] + X->w_order);
  HIP_OK(hipMemcpyAsync(out, order + t0, cnt * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return TDG_OK;
}

// Internal (host-side index replay in the tests): the matrix-core evaluation
// tables of degree p and the moment-phase chunk.  info[22] = {ev_nl, ev_nat,
// ev_nks[0..7], M, W1 doubles, mpch[p], moff[p] (-1: the default regions),
// ev_nkv[0..7]}.
int tdg_debug_eval_tables(const tdg_ctx* X, int32_t p, int32_t* info, int32_t* ev_ab, int32_t* ev_ex) {
  if (!X || !info) return fail(TDG_EINVAL, "NULL argument");
  if (p < 1 || p > X->opts.p_max) return fail(TDG_EINVAL, "p out of range");
  const Table& t = X->tabs[p];
  info[0] = t.ev_nl;
  info[1] = t.ev_nat;
  for (int i = 0; i < 8; ++i) info[2 + i] = t.ev_nks[i];
  info[10] = t.M;
  info[11] = X->lp.off_fg - X->lp.off_W1;
  info[12] = X->lp.mpch[p];
  info[13] = X->lp.moff[p];
  for (int i = 0; i < 8; ++i) info[14 + i] = t.ev_nkv[i];
  if (ev_ab) std::copy(t.ev_ab.begin(), t.ev_ab.end(), ev_ab);
  if (ev_ex) std::copy(t.ev_ex.begin(), t.ev_ex.end(), ev_ex);
  return TDG_OK;
}

// Internal (host-side table checks in the tests): the field and U tables of
// degree p as built.  info[5] = {M, NW, n, nnz of the field rows, nnz of the U
// rows}; expo[M (n+1)] the exponents (t first) of the monomials, fo_ptr[NW (n+1)
// + 1] / fo_idx / fo_coef the rows (function j, component v, sigma_1..n) and
// u_ptr[NW + 1] / u_idx / u_coef those of U_j.  Arrays are nullable.
int tdg_debug_field_tables(const tdg_ctx* X, int32_t p, int32_t* info, int32_t* expo, int32_t* fo_ptr,
                           int32_t* fo_idx, double* fo_coef, int32_t* u_ptr, int32_t* u_idx, double* u_coef) {
  if (!X || !info) return fail(TDG_EINVAL, "NULL argument");
  if (p < 1 || p > X->opts.p_max) return fail(TDG_EINVAL, "p out of range");
  const Table& t = X->tabs[p];
  info[0] = t.M;
  info[1] = t.NW;
  info[2] = X->topo.n;
  info[3] = (int32_t)t.fo_idx.size();
  info[4] = (int32_t)t.u_idx.size();
  if (expo) std::copy(t.expo.begin(), t.expo.end(), expo);
  if (fo_ptr) std::copy(t.fo_ptr.begin(), t.fo_ptr.end(), fo_ptr);
  if (fo_idx) std::copy(t.fo_idx.begin(), t.fo_idx.end(), fo_idx);
  if (fo_coef) std::copy(t.fo_coef.begin(), t.fo_coef.end(), fo_coef);
  if (u_ptr) std::copy(t.u_ptr.begin(), t.u_ptr.end(), u_ptr);
  if (u_idx) std::copy(t.u_idx.begin(), t.u_idx.end(), u_idx);
  if (u_coef) std::copy(t.u_coef.begin(), t.u_coef.end(), u_coef);
  return TDG_OK;
}

void trefftz_destroy(tdg_ctx* X) {
  if (X) drop_graph(X);
  delete X;
}

}  // extern "C"
