// Per-tent Trefftz-DG solve on gfx950: one workgroup per tent, all tents of a
// layer in one launch (tents of a layer share no element, Sec. 2.2).
//
// For the tent at vertex V with bottom front phi_old and top front phi_new
// (phi_new = phi_old + (t_top - t_bot) lambda_V on each patch element):
//   1. gather the patch: vertex coordinates, front heights, grad phi, speeds;
//      group the elements by speed (Sec. 4.2)
//   2. per speed group, shift and scale the c = 1 Trefftz basis (Remark 3.1):
//      xh = (x - X_V)/h, th = c (t - t_mid)/h with h the anisotropic diameter
//      (eq. 3.3) of the tent; v = c dU/dth, sigma = -grad_xh U, U_j = h Uhat_j
//   3. top facets (eq. 4.1 written on the graph t = phi(x)):
//        A += sum_q w [c^-2 v_i v_j + s_i.s_j - (v_i s_j + v_j s_i).grad phi_new]
//      computed as Psi^T Psi with Psi = sqrt(w) D^(1/2) B Phi, where
//      G = [[c^-2, -g^T], [-g, I]] = B^T D B, B = [[1, 0], [-g, I]],
//      D = diag(c^-2 - |g|^2, I) (positive on space-like facets)
//   4. bottom facets: rhs_i += sum_q w Phi_i(bottom)^T G_old u_bot
//      and the recovery row of U (Sec. 5): mean of U over the bottom
//   5. Dirichlet faces: A_ij += w v_i (alpha v_j + s_j.n), rhs_i += w g_D (alpha v_i - s_i.n)
//   6. speed interfaces: centred fluxes with penalties (Sec. 4.2)
//   7. LU with partial pivoting, back substitution, U constants
//   8. evaluate (v, sigma, U) at the top points and overwrite the stored values;
//      tau_V = t_top
#include <hip/hip_runtime.h>

#include "tdg_internal.h"

namespace tdg {

namespace {

template <int NS>
struct El {
  // offsets inside one patch-element record
  static constexpr int X = 0;                       // (NS+1) vertices x NS coords
  static constexpr int TAU = (NS + 1) * NS;         // NS+1 heights
  static constexpr int GOLD = TAU + NS + 1;         // NS
  static constexpr int GNEW = GOLD + NS;            // NS
  static constexpr int C = GNEW + NS;
  static constexpr int DET = C + 1;
  static constexpr int GRP = DET + 1;
  static constexpr int LV = GRP + 1;
  static constexpr int E = LV + 1;
  static constexpr int SIZE = E + 1;
};

__device__ inline void atomic_max_nonneg(double* addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

// Monomials t^k x^alpha of one point (thread-private column of mono).
__device__ inline void eval_mono(const TableDesc& T, int count, double* mono, int PCH, int pt, const double* var) {
  mono[pt] = 1.0;
  for (int i = 1; i < count; ++i) mono[i * PCH + pt] = mono[T.parent[i] * PCH + pt] * var[T.var[i]];
}

// Fields (vhat, sigmahat) of non-constant basis function j at one point.
template <int NS>
__device__ inline void eval_fields(const TableDesc& T, int j, const double* mono, int PCH, int pt, double* out) {
#pragma unroll
  for (int comp = 0; comp <= NS; ++comp) {
    double acc = 0.0;
    const int r = j * (NS + 1) + comp;
    for (int e = T.fo_ptr[r]; e < T.fo_ptr[r + 1]; ++e) acc += T.fo_coef[e] * mono[T.fo_idx[e] * PCH + pt];
    out[comp] = acc;
  }
}

__device__ inline double eval_u(const TableDesc& T, int j, const double* mono, int PCH, int pt) {
  double acc = 0.0;
  for (int e = T.u_ptr[j]; e < T.u_ptr[j + 1]; ++e) acc += T.u_coef[e] * mono[T.u_idx[e] * PCH + pt];
  return acc;
}

// C[i][j] += sum_k L[k][i] R[k][j] for i, j < NW over nrow rows (LDS, row stride NWP)
__device__ inline void acc_block(double* A, int lda, int r0, int c0, const double* L, const double* R, int nrow,
                                 int NWP, int NW) {
  for (int idx = threadIdx.x; idx < NW * NW; idx += blockDim.x) {
    const int i = idx / NW, j = idx % NW;
    double acc = 0.0;
    for (int k = 0; k < nrow; ++k) acc += L[k * NWP + i] * R[k * NWP + j];
    A[(r0 + i) * lda + c0 + j] += acc;
  }
}

}  // namespace

template <int NS>
__global__ __launch_bounds__(kBlock) void tent_layer_kernel(KParams P, LdsPlan L, int t0) {
  extern __shared__ double lds[];
  double* A = lds + L.off_A;
  double* xs = lds + L.off_x;
  double* mono = lds + L.off_mono;
  double* W1 = lds + L.off_W1;
  double* W2 = lds + L.off_W2;
  double* EL = lds + L.off_el;
  double* MS = lds + L.off_misc;
  // misc layout
  double* gc = MS;                    // kMaxGroups speeds
  double* gh = gc + kMaxGroups;       // kMaxGroups diameters
  double* A00 = gh + kMaxGroups;      // kMaxGroups
  double* r0 = A00 + kMaxGroups;      // kMaxGroups
  double* a0 = r0 + kMaxGroups;       // kMaxGroups
  double* fsc = a0 + kMaxGroups;      // face scalars: measure, normal, simplex vertices (24)
  double* A0 = fsc + 24;              // kMaxGroups x NWP
  __shared__ int s_m, s_piv, s_err;

  const int tid = threadIdx.x;
  const int tent = t0 + blockIdx.x;
  const int V = P.tent_V[tent];
  const double tb = P.tent_tb[tent], tt = P.tent_tt[tent];
  const double tmid = 0.5 * (tb + tt);
  const double dt = tt - tb;
  const int p = P.p_per_tent ? (int)P.p_per_tent[tent] : P.pmax;
  const int pb = P.v2e_ptr[V];
  const int npatch = P.v2e_ptr[V + 1] - pb;
  const int Q = P.Q;
  const int PCH = L.PCH;
  const int NWP = L.NWP;
  const int lda = L.lda;
  const int ELS = L.ELS;
  if (p < 1 || p > P.pmax || npatch > L.maxpatch) {
    if (tid == 0) atomicOr(P.status, p < 1 || p > P.pmax ? kStatSize : kStatPatch);
    return;
  }
  const TableDesc T = P.tab[p];
  const int NW = T.NW;
  const double* XV = P.coords + (size_t)V * NS;

  // ---- 1. patch records -------------------------------------------------------
  for (int i = tid; i < npatch; i += blockDim.x) {
    const int e = P.v2e[pb + i];
    double* R = EL + i * ELS;
    const int* vs = P.elems + (size_t)e * (NS + 1);
    const double* gl = P.grad_lam + (size_t)e * (NS + 1) * NS;
    int lV = 0;
    double go[NS];
#pragma unroll
    for (int d = 0; d < NS; ++d) go[d] = 0.0;
#pragma unroll
    for (int k = 0; k <= NS; ++k) {
      const int v = vs[k];
      const double tk = P.tau[v];
      R[El<NS>::TAU + k] = tk;
#pragma unroll
      for (int d = 0; d < NS; ++d) {
        R[El<NS>::X + k * NS + d] = P.coords[(size_t)v * NS + d];
        go[d] += tk * gl[k * NS + d];
      }
      if (v == V) lV = k;
    }
#pragma unroll
    for (int d = 0; d < NS; ++d) {
      R[El<NS>::GOLD + d] = go[d];
      R[El<NS>::GNEW + d] = go[d] + dt * gl[lV * NS + d];
    }
    R[El<NS>::C] = P.c[e];
    R[El<NS>::DET] = P.absdet[e];
    R[El<NS>::LV] = (double)lV;
    R[El<NS>::E] = (double)e;
  }
  if (tid < kMaxGroups) {
    gh[tid] = 0.0;
    A00[tid] = 0.0;
    r0[tid] = 0.0;
  }
  if (tid == 0) s_err = 0;
  __syncthreads();
  if (tid == 0) {
    int m = 0;
    for (int i = 0; i < npatch; ++i) {
      const double ce = EL[i * ELS + El<NS>::C];
      int g = -1;
      for (int r = 0; r < m; ++r)
        if (gc[r] == ce) g = r;
      if (g < 0) {
        if (m == kMaxGroups) {
          s_err = kStatGroups;
          g = 0;
        } else {
          gc[m] = ce;
          g = m++;
        }
      }
      EL[i * ELS + El<NS>::GRP] = (double)g;
    }
    s_m = m;
  }
  __syncthreads();
  const int m = s_m;
  const int S = m * NW;
  if (s_err || S > L.S) {
    if (tid == 0) atomicOr(P.status, s_err ? s_err : kStatSize);
    return;
  }

  // ---- 2. anisotropic diameter per group over the tent's space-time vertices ---
  {
    const int nvert = npatch * (NS + 1) + 1;  // element vertices (repeats allowed) + top of V
    const long long npair = (long long)nvert * (nvert - 1) / 2;
    double hloc[kMaxGroups];
    for (int r = 0; r < kMaxGroups; ++r) hloc[r] = 0.0;
    for (long long pi = tid; pi < npair; pi += blockDim.x) {
      // unrank pair (a, b), a < b
      int a = 0;
      long long rem = pi;
      while (rem >= nvert - 1 - a) {
        rem -= nvert - 1 - a;
        ++a;
      }
      const int b = a + 1 + (int)rem;
      double xa[NS], xb[NS], ta, tbv;
      if (a == nvert - 1) {
        for (int d = 0; d < NS; ++d) xa[d] = XV[d];
        ta = tt;
      } else {
        const double* R = EL + (a / (NS + 1)) * ELS;
        for (int d = 0; d < NS; ++d) xa[d] = R[El<NS>::X + (a % (NS + 1)) * NS + d];
        ta = R[El<NS>::TAU + a % (NS + 1)];
      }
      if (b == nvert - 1) {
        for (int d = 0; d < NS; ++d) xb[d] = XV[d];
        tbv = tt;
      } else {
        const double* R = EL + (b / (NS + 1)) * ELS;
        for (int d = 0; d < NS; ++d) xb[d] = R[El<NS>::X + (b % (NS + 1)) * NS + d];
        tbv = R[El<NS>::TAU + b % (NS + 1)];
      }
      double dx2 = 0.0;
      for (int d = 0; d < NS; ++d) dx2 += (xa[d] - xb[d]) * (xa[d] - xb[d]);
      const double dtt = ta - tbv;
      for (int r = 0; r < m; ++r) hloc[r] = fmax(hloc[r], sqrt(dx2 + gc[r] * gc[r] * dtt * dtt));
    }
    for (int r = 0; r < m; ++r) atomic_max_nonneg(&gh[r], hloc[r]);
  }
  // zero the system
  for (int i = tid; i < S * lda; i += blockDim.x) A[i] = 0.0;
  for (int i = tid; i < kMaxGroups * NWP; i += blockDim.x) A0[i] = 0.0;
  __syncthreads();

  const int parts = blockDim.x / PCH;
  const int pt = tid % PCH;
  const int part = tid / PCH;
  double* PV = W2;                       // PCH x (NS+1): (th, xh_1..xh_n)
  double* PD = W2 + PCH * (NS + 1);      // PCH x (NS+2): bottom data d_0..d_n, w*U_b
  double* PWt = PD + PCH * (NS + 2);     // PCH weights

  // ---- 3./4. top Gram, bottom right-hand side, U recovery rows ------------------
  for (int i = 0; i < npatch; ++i) {
    const double* R = EL + i * ELS;
    const int r = (int)R[El<NS>::GRP];
    const double ce = R[El<NS>::C];
    const double hr = gh[r];
    const int lV = (int)R[El<NS>::LV];
    const int e = (int)R[El<NS>::E];
    const double det = R[El<NS>::DET];
    const double ic2 = 1.0 / (ce * ce);
    double gn[NS], go[NS], gn2 = 0.0;
    for (int d = 0; d < NS; ++d) {
      gn[d] = R[El<NS>::GNEW + d];
      go[d] = R[El<NS>::GOLD + d];
      gn2 += gn[d] * gn[d];
    }
    const double sD = ic2 - gn2;  // > 0 on a space-like top facet
    const double* st = P.state + (size_t)e * (NS + 2) * Q;
    for (int q0 = 0; q0 < Q; q0 += PCH) {
      // top points
      if (tid < PCH) {
        const int q = q0 + pt;
        double x[NS], phi = 0.0, w = 0.0;
        for (int d = 0; d < NS; ++d) x[d] = 0.0;
        if (q < Q) {
          const double* lam = P.lam_ref + (size_t)q * (NS + 1);
          for (int k = 0; k <= NS; ++k) {
            phi += lam[k] * R[El<NS>::TAU + k];
            for (int d = 0; d < NS; ++d) x[d] += lam[k] * R[El<NS>::X + k * NS + d];
          }
          phi += lam[lV] * dt;
          w = P.w_ref[q] * det;
        }
        PV[pt * (NS + 1)] = ce * (phi - tmid) / hr;
        for (int d = 0; d < NS; ++d) PV[pt * (NS + 1) + 1 + d] = (x[d] - XV[d]) / hr;
        PWt[pt] = w;
        eval_mono(T, T.M1, mono, PCH, pt, PV + pt * (NS + 1));
      }
      __syncthreads();
      {
        const double w = PWt[pt];
        const double sw = sqrt(w), swD = sqrt(w * sD);
        for (int j = part; j < NW; j += parts) {
          double f[NS + 1];
          eval_fields<NS>(T, j, mono, PCH, pt, f);
          const double v = ce * f[0];
          double* row = W1 + (size_t)pt * (NS + 1) * NWP + j;
          row[0] = swD * v;
          for (int d = 0; d < NS; ++d) row[(1 + d) * NWP] = sw * (f[1 + d] - gn[d] * v);
        }
      }
      __syncthreads();
      acc_block(A, lda, r * NW, r * NW, W1, W1, PCH * (NS + 1), NWP, NW);
      __syncthreads();
      // bottom points
      if (tid < PCH) {
        const int q = q0 + pt;
        double x[NS], phi = 0.0, w = 0.0;
        for (int d = 0; d < NS; ++d) x[d] = 0.0;
        double dd[NS + 2];
        for (int k = 0; k < NS + 2; ++k) dd[k] = 0.0;
        if (q < Q) {
          const double* lam = P.lam_ref + (size_t)q * (NS + 1);
          for (int k = 0; k <= NS; ++k) {
            phi += lam[k] * R[El<NS>::TAU + k];
            for (int d = 0; d < NS; ++d) x[d] += lam[k] * R[El<NS>::X + k * NS + d];
          }
          w = P.w_ref[q] * det;
          const double vb = st[q];
          double sg = 0.0;
          for (int d = 0; d < NS; ++d) sg += st[(1 + d) * Q + q] * go[d];
          dd[0] = w * (ic2 * vb - sg);
          for (int d = 0; d < NS; ++d) dd[1 + d] = w * (st[(1 + d) * Q + q] - vb * go[d]);
          dd[NS + 1] = w * st[(NS + 1) * Q + q];
        }
        PV[pt * (NS + 1)] = ce * (phi - tmid) / hr;
        for (int d = 0; d < NS; ++d) PV[pt * (NS + 1) + 1 + d] = (x[d] - XV[d]) / hr;
        for (int k = 0; k < NS + 2; ++k) PD[pt * (NS + 2) + k] = dd[k];
        PWt[pt] = w;
        eval_mono(T, T.M, mono, PCH, pt, PV + pt * (NS + 1));
      }
      __syncthreads();
      {
        const double w = PWt[pt];
        for (int j = part; j < NW; j += parts) {
          double f[NS + 1];
          eval_fields<NS>(T, j, mono, PCH, pt, f);
          double acc = ce * f[0] * PD[pt * (NS + 2)];
          for (int d = 0; d < NS; ++d) acc += f[1 + d] * PD[pt * (NS + 2) + 1 + d];
          W1[pt * NWP + j] = acc;
          W1[(PCH + pt) * NWP + j] = w * hr * eval_u(T, j, mono, PCH, pt);
        }
      }
      __syncthreads();
      for (int j = tid; j < NW; j += blockDim.x) {
        double acc = 0.0, acc0 = 0.0;
        for (int k = 0; k < PCH; ++k) {
          acc += W1[k * NWP + j];
          acc0 += W1[(PCH + k) * NWP + j];
        }
        A[(r * NW + j) * lda + S] += acc;
        A0[r * NWP + j] += acc0;
      }
      if (tid == blockDim.x - 1) {
        double sw = 0.0, su = 0.0;
        for (int k = 0; k < PCH; ++k) {
          sw += PWt[k];
          su += PD[k * (NS + 2) + NS + 1];
        }
        A00[r] += sw;
        r0[r] += su;
      }
      __syncthreads();
    }
  }

  // ---- 5./6. time-like faces above facets containing V --------------------------
  const int nbf = P.vb_ptr[V + 1] - P.vb_ptr[V];
  const int nif = P.vi_ptr[V + 1] - P.vi_ptr[V];
  for (int f = 0; f < nbf + nif; ++f) {
    const bool dir = f < nbf;
    int e1, k1, e2 = -1;
    if (dir) {
      e1 = P.vb[2 * (P.vb_ptr[V] + f)];
      k1 = P.vb[2 * (P.vb_ptr[V] + f) + 1];
    } else {
      const int* q4 = P.vi + 4 * (P.vi_ptr[V] + f - nbf);
      e1 = q4[0];
      k1 = q4[1];
      e2 = q4[2];
    }
    // face simplex: (X_V, tb), (X_V, tt), (X_W, tau_W) for W in facet \ {V}
    if (tid == 0) {
      const int* vs = P.elems + (size_t)e1 * (NS + 1);
      double Pv[NS + 1][NS + 1];
      for (int d = 0; d < NS; ++d) {
        Pv[0][d] = XV[d];
        Pv[1][d] = XV[d];
      }
      Pv[0][NS] = tb;
      Pv[1][NS] = tt;
      int c = 2;
      for (int k = 0; k <= NS; ++k) {
        const int w = vs[k];
        if (k == k1 || w == V) continue;
        for (int d = 0; d < NS; ++d) Pv[c][d] = P.coords[(size_t)w * NS + d];
        Pv[c][NS] = P.tau[w];
        ++c;
      }
      // Gram of the edge vectors E_i = P_i - P_0, i = 1..NS
      double E[NS][NS + 1], G[NS][NS];
      for (int i = 0; i < NS; ++i)
        for (int d = 0; d <= NS; ++d) E[i][d] = Pv[i + 1][d] - Pv[0][d];
      for (int i = 0; i < NS; ++i)
        for (int j = 0; j < NS; ++j) {
          double s = 0.0;
          for (int d = 0; d <= NS; ++d) s += E[i][d] * E[j][d];
          G[i][j] = s;
        }
      double detG;
      if (NS == 1)
        detG = G[0][0];
      else if (NS == 2)
        detG = G[0][0] * G[1][1] - G[0][1] * G[1][0];
      else
        detG = G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1]) - G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0]) +
               G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]);
      fsc[0] = sqrt(fmax(detG, 0.0));
      const double* gl = P.grad_lam + ((size_t)e1 * (NS + 1) + k1) * NS;
      double nn = 0.0;
      for (int d = 0; d < NS; ++d) nn += gl[d] * gl[d];
      nn = sqrt(nn);
      for (int d = 0; d < NS; ++d) fsc[1 + d] = -gl[d] / nn;
      for (int i = 0; i <= NS; ++i)
        for (int d = 0; d <= NS; ++d) fsc[4 + i * (NS + 1) + d] = Pv[i][d];
      // groups of the two sides
      int g1 = 0, g2 = 0;
      for (int i = 0; i < npatch; ++i) {
        const int e = (int)EL[i * ELS + El<NS>::E];
        if (e == e1) g1 = (int)EL[i * ELS + El<NS>::GRP];
        if (e == e2) g2 = (int)EL[i * ELS + El<NS>::GRP];
      }
      s_piv = g1 * 16 + g2;
    }
    __syncthreads();
    const double meas = fsc[0];
    double nrm[NS];
    for (int d = 0; d < NS; ++d) nrm[d] = fsc[1 + d];
    const int ga = s_piv / 16, gb = s_piv % 16;
    const long long goff = P.bpt_off[tent] + (long long)f * Q;
    for (int q0 = 0; q0 < Q; q0 += PCH) {
      const int nside = dir ? 1 : 2;
      for (int side = 0; side < nside; ++side) {
        const int r = side == 0 ? ga : gb;
        const double cr = gc[r], hr = gh[r];
        if (tid < PCH) {
          const int q = q0 + pt;
          double y[NS + 1];
          for (int d = 0; d <= NS; ++d) y[d] = 0.0;
          double w = 0.0, g = 0.0;
          if (q < Q) {
            const double* lam = P.lam_ref + (size_t)q * (NS + 1);
            for (int k = 0; k <= NS; ++k)
              for (int d = 0; d <= NS; ++d) y[d] += lam[k] * fsc[4 + k * (NS + 1) + d];
            w = P.w_ref[q] * meas;
            if (dir) g = P.gD[goff + q];
          } else {
            for (int d = 0; d < NS; ++d) y[d] = XV[d];
            y[NS] = tmid;
          }
          PV[pt * (NS + 1)] = cr * (y[NS] - tmid) / hr;
          for (int d = 0; d < NS; ++d) PV[pt * (NS + 1) + 1 + d] = (y[d] - XV[d]) / hr;
          PWt[pt] = w;
          PD[pt] = g;
          eval_mono(T, T.M1, mono, PCH, pt, PV + pt * (NS + 1));
        }
        __syncthreads();
        {
          const double w = PWt[pt], sw = sqrt(w), g = PD[pt];
          for (int j = part; j < NW; j += parts) {
            double fl[NS + 1];
            eval_fields<NS>(T, j, mono, PCH, pt, fl);
            const double v = cr * fl[0];
            double sn = 0.0;
            for (int d = 0; d < NS; ++d) sn += fl[1 + d] * nrm[d];
            if (dir) {
              W1[pt * NWP + j] = sw * v;
              W1[(PCH + pt) * NWP + j] = sw * (P.alpha * v + sn);
              W1[(2 * PCH + pt) * NWP + j] = w * g * (P.alpha * v - sn);
            } else {
              W1[((2 * side) * PCH + pt) * NWP + j] = sw * v;
              W1[((2 * side + 1) * PCH + pt) * NWP + j] = sw * sn;
            }
          }
        }
        __syncthreads();
      }
      if (dir) {
        acc_block(A, lda, ga * NW, ga * NW, W1, W1 + PCH * NWP, PCH, NWP, NW);
        for (int j = tid; j < NW; j += blockDim.x) {
          double acc = 0.0;
          for (int k = 0; k < PCH; ++k) acc += W1[(2 * PCH + k) * NWP + j];
          A[(ga * NW + j) * lda + S] += acc;
        }
      } else {
        // test in group b (sign sb), trial in group a (sign sa):
        // w_i (alpha sa sb v_j + sb/2 s_j.n) + (tau_i.n)(sb/2 v_j + beta sa sb s_j.n)
        for (int blk = 0; blk < 4; ++blk) {
          const int sa_i = blk / 2, sb_i = blk % 2;  // side index of trial / test
          const double sa = sa_i ? -1.0 : 1.0, sb = sb_i ? -1.0 : 1.0;
          const int gA = sa_i ? gb : ga, gB = sb_i ? gb : ga;
          const double* Va = W1 + (2 * sa_i) * PCH * NWP;
          const double* Na = W1 + (2 * sa_i + 1) * PCH * NWP;
          const double* Vb = W1 + (2 * sb_i) * PCH * NWP;
          const double* Nb = W1 + (2 * sb_i + 1) * PCH * NWP;
          for (int idx = tid; idx < NW * NW; idx += blockDim.x) {
            const int ii = idx / NW, jj = idx % NW;
            double acc = 0.0;
            for (int k = 0; k < PCH; ++k) {
              const double va = Va[k * NWP + jj], na = Na[k * NWP + jj];
              acc += Vb[k * NWP + ii] * (P.alpha * sa * sb * va + 0.5 * sb * na) +
                     Nb[k * NWP + ii] * (0.5 * sb * va + P.beta * sa * sb * na);
            }
            A[(gB * NW + ii) * lda + gA * NW + jj] += acc;
          }
        }
      }
      __syncthreads();
    }
  }

  // ---- 7. LU with partial pivoting on the augmented matrix -----------------------
  for (int k = 0; k < S; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bi = S;
      for (int rr = k + tid; rr < S; rr += 64) {
        const double v = fabs(A[rr * lda + k]);
        if (v > best) {
          best = v;
          bi = rr;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_down(best, off, 64);
        const int oi = __shfl_down(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) s_piv = bi;
    }
    __syncthreads();
    const int pr = s_piv;
    if (pr != k)
      for (int j = k + tid; j <= S; j += blockDim.x) {
        const double t = A[k * lda + j];
        A[k * lda + j] = A[pr * lda + j];
        A[pr * lda + j] = t;
      }
    __syncthreads();
    const double piv = A[k * lda + k];
    if (piv == 0.0) {
      if (tid == 0) s_err = kStatSingular;
      break;
    }
    for (int i = k + 1 + tid; i < S; i += blockDim.x) A[i * lda + k] /= piv;
    __syncthreads();
    const int nr = S - k - 1, nc = S - k;
    for (int idx = tid; idx < nr * nc; idx += blockDim.x) {
      const int i = k + 1 + idx / nc, j = k + 1 + idx % nc;
      A[i * lda + j] -= A[i * lda + k] * A[k * lda + j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (s_err) {
    if (tid == 0) atomicOr(P.status, s_err);
    return;
  }
  for (int k = S - 1; k >= 0; --k) {
    if (tid == 0) xs[k] = A[k * lda + S] / A[k * lda + k];
    __syncthreads();
    const double xk = xs[k];
    for (int i = tid; i < k; i += blockDim.x) A[i * lda + S] -= A[i * lda + k] * xk;
    __syncthreads();
  }
  // U constants (Sec. 5): mean of U over the bottom matches the incoming mean
  if (tid < m) {
    double s = r0[tid];
    for (int j = 0; j < NW; ++j) s -= A0[tid * NWP + j] * xs[tid * NW + j];
    a0[tid] = P.recover_U ? s / A00[tid] : 0.0;
  }
  __syncthreads();

  // ---- 8. top values overwrite the stored values -------------------------------
  double* cm = W1;                 // (NS+1) x M1: field coefficients contracted with x
  double* cu = W1 + (NS + 1) * T.M1;  // M: U coefficients contracted with x
  for (int r = 0; r < m; ++r) {
    for (int i = tid; i < (NS + 1) * T.M1 + T.M; i += blockDim.x) cm[i] = 0.0;
    __syncthreads();
    if (tid <= NS) {
      const int comp = tid;
      for (int j = 0; j < NW; ++j) {
        const double xj = xs[r * NW + j];
        const int row = j * (NS + 1) + comp;
        for (int e = T.fo_ptr[row]; e < T.fo_ptr[row + 1]; ++e) cm[comp * T.M1 + T.fo_idx[e]] += T.fo_coef[e] * xj;
      }
    } else if (tid == NS + 1) {
      for (int j = 0; j < NW; ++j) {
        const double xj = xs[r * NW + j] * gh[r];
        for (int e = T.u_ptr[j]; e < T.u_ptr[j + 1]; ++e) cu[T.u_idx[e]] += T.u_coef[e] * xj;
      }
    }
    __syncthreads();
    const double cr = gc[r], hr = gh[r];
    for (int i = 0; i < npatch; ++i) {
      const double* R = EL + i * ELS;
      if ((int)R[El<NS>::GRP] != r) continue;
      const int lV = (int)R[El<NS>::LV];
      const int e = (int)R[El<NS>::E];
      double* st = P.state + (size_t)e * (NS + 2) * Q;
      for (int q0 = 0; q0 < Q; q0 += PCH) {
        if (tid < PCH) {
          const int q = q0 + pt;
          double x[NS], phi = 0.0;
          for (int d = 0; d < NS; ++d) x[d] = 0.0;
          if (q < Q) {
            const double* lam = P.lam_ref + (size_t)q * (NS + 1);
            for (int k = 0; k <= NS; ++k) {
              phi += lam[k] * R[El<NS>::TAU + k];
              for (int d = 0; d < NS; ++d) x[d] += lam[k] * R[El<NS>::X + k * NS + d];
            }
            phi += lam[lV] * dt;
          }
          PV[pt * (NS + 1)] = cr * (phi - tmid) / hr;
          for (int d = 0; d < NS; ++d) PV[pt * (NS + 1) + 1 + d] = (x[d] - XV[d]) / hr;
          eval_mono(T, T.M, mono, PCH, pt, PV + pt * (NS + 1));
          if (q < Q) {
            double out[NS + 2];
            for (int comp = 0; comp <= NS; ++comp) {
              double acc = 0.0;
              for (int k = 0; k < T.M1; ++k) acc += cm[comp * T.M1 + k] * mono[k * PCH + pt];
              out[comp] = acc;
            }
            out[0] *= cr;
            double u = a0[r];
            for (int k = 0; k < T.M; ++k) u += cu[k] * mono[k * PCH + pt];
            out[NS + 1] = u;
            bool bad = false;
            for (int comp = 0; comp < NS + 2; ++comp) {
              st[comp * Q + q] = out[comp];
              bad = bad || !isfinite(out[comp]);
            }
            if (bad) atomicOr(P.status, kStatNan);
          }
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) P.tau[V] = tt;
}

int launch_layer(const KParams& P, const LdsPlan& L, int t0, int count, void* stream_) {
  hipStream_t stream = (hipStream_t)stream_;
  if (count <= 0) return 0;
  dim3 grid(count), block(kBlock);
  size_t shm = (size_t)L.total * sizeof(double);
  switch (P.n) {
    case 1:
      hipLaunchKernelGGL(tent_layer_kernel<1>, grid, block, shm, stream, P, L, t0);
      break;
    case 2:
      hipLaunchKernelGGL(tent_layer_kernel<2>, grid, block, shm, stream, P, L, t0);
      break;
    default:
      hipLaunchKernelGGL(tent_layer_kernel<3>, grid, block, shm, stream, P, L, t0);
      break;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int set_kernel_smem_limit(int n, size_t bytes) {
  hipError_t e;
  switch (n) {
    case 1:
      e = hipFuncSetAttribute((const void*)tent_layer_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      break;
    case 2:
      e = hipFuncSetAttribute((const void*)tent_layer_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      break;
    default:
      e = hipFuncSetAttribute((const void*)tent_layer_kernel<3>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      break;
  }
  return e == hipSuccess ? 0 : -1;
}

}  // namespace tdg
