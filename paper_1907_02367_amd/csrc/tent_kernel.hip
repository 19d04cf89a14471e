// Per-tent Trefftz-DG solve on gfx950: one workgroup (4 waves) per tent, all
// tents of a layer in one launch (tents of a layer share no element, Sec. 2.2).
//
// For the tent at vertex V with bottom front phi_old and top front phi_new
// (phi_new = phi_old + (t_top - t_bot) lambda_V on each patch element):
//   1. gather the patch (coordinates, front heights, grad phi, speeds); group
//      the elements by speed (Sec. 4.2); anisotropic diameter per group (eq. 3.3)
//   2. per group, the c = 1 Trefftz basis is shifted and scaled (Remark 3.1):
//      xh = (x - X_V)/h, th = c (t - t_mid)/h; v = c dU/dth, sigma = -grad_xh U,
//      U_j = h Uhat_j.  The points of all elements of the group form one list,
//      processed in chunks of PCH points:
//        - top facets (eq. 4.1 on the graph t = phi_new(x)):
//              A += sum_q w Phi^T G_new Phi = Psi^T Psi,  Psi = sqrt(w) D^(1/2) B Phi,
//          G = [[c^-2, -g^T], [-g, I]] = B^T D B, B = [[1, 0], [-g, I]],
//          D = diag(c^-2 - |g|^2, I) (positive on space-like facets).
//          The Gram Psi^T Psi runs on the FP64 matrix cores (16x16x4 tiles).
//        - bottom facets: rhs_i += sum_q w Phi_i(bottom)^T G_old u_bot, and the
//          U recovery row (Sec. 5): the mean of U over the bottom facets.
//   3. Dirichlet faces: A_ij += w v_i (alpha v_j + s_j.n), rhs_i += w g_D (alpha v_i - s_i.n);
//      speed interfaces: centred fluxes with penalties (Sec. 4.2).
//   4. LU: one wave with rows in registers and diagonal pivots for systems up
//      to 32 unknowns; the whole workgroup with partial pivoting otherwise, back substitution, U constants.
//   5. optional indicator: energy of the jump between the new solution and the
//      incoming trace on the bottom facets (a term of the tent's energy
//      balance); a tent solved below p_max whose indicator exceeds the
//      tolerance is solved again one degree higher (up to p_max) before
//      anything is written
//   6. (v, sigma, U) at the top points overwrite the stored values; tau_V = t_top.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "tdg_internal.h"

namespace tdg {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kIRMax = 6;  // refinement steps of the mixed-precision solve

template <int NS>
struct El {
  // offsets inside one patch-element record (doubles)
  static constexpr int X = 0;                // (NS+1) vertices x NS coordinates
  static constexpr int TAU = (NS + 1) * NS;  // NS+1 front heights
  static constexpr int GOLD = TAU + NS + 1;  // grad phi_old
  static constexpr int GNEW = GOLD + NS;     // grad phi_new
  static constexpr int C = GNEW + NS;
  static constexpr int DET = C + 1;
  static constexpr int GRP = DET + 1;
  static constexpr int LV = GRP + 1;
  static constexpr int E = LV + 1;
  static constexpr int SIZE = E + 1;
};

__device__ inline void atomic_max_nonneg(double* addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

// load from global memory through a global (not flat) address: flat loads also
// count against the LDS wait counter, so every later LDS wait would wait for them
__device__ inline double gload(const double* p) {
  return *(const __attribute__((address_space(1))) double*)p;
}

// Sums of a and b over the workgroup (lanes by butterflies, then the waves in
// order; deterministic): every thread returns the totals.  scratch: 2 doubles per
// wave of LDS, free for the call; the call starts and ends with a barrier.
__device__ inline void block_sum2(double& a, double& b, double* scratch) {
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) {
    scratch[2 * wave] = a;
    scratch[2 * wave + 1] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  for (int w = 0; w < (int)blockDim.x / 64; ++w) {
    a += scratch[2 * w];
    b += scratch[2 * w + 1];
  }
  __syncthreads();
}

// A double from another lane of the same row of 16 lanes by a DPP control
// (register-to-register, no LDS): the two 32-bit halves move separately.
template <int CTRL>
__device__ inline double dpp_row(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over each row of 16 lanes, every lane of the row receiving it: the pairs
// of the butterfly over lane bits 0..3 (quad_perm [1,0,3,2] and [2,3,0,1],
// then the half-row and row mirrors, which meet lanes holding the same partial
// sums as lane ^ 4 and lane ^ 8), so the additions are those of the butterfly.
__device__ inline double row16_sum(double v) {
  v += dpp_row<0xB1>(v);
  v += dpp_row<0x4E>(v);
  v += dpp_row<0x141>(v);
  v += dpp_row<0x140>(v);
  return v;
}

// ordering of LDS accesses inside one wave (no workgroup barrier needed)
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Table of one degree, possibly staged in LDS (see TableDesc).
struct Tab {
  const int* ue_ptr;
  const int* ue_idx;
  const double* ue_coef;
  const int* tr_ptr;
  const int* tr_j;
  const double* tr_coef;
  const int* expo;  // M*(NS+1) exponents (k, alpha)
  // moment mode (global memory): sparse fields per (function, component), U rows,
  // moment monomials and the product index
  const int* fo_ptr;
  const int* fo_idx;
  const double* fo_coef;
  const int* u_ptr;
  const int* u_idx;
  const double* u_coef;
  const int* expo2;
  const int* K2;
  const int* task2;
  const int* task1;
  int NW, M, M1, M2, ntask2, ntask1;
};

// Monomials of points [0, npt) from their coordinates var[pt*(NS+1) + v]
// (v = 0: th, v >= 1: xh_v): first the powers, then each monomial as a product
// of powers (flat parallel over (point, monomial)).  mono has row stride ld.
template <int NS>
__device__ inline void monomials(const Tab& T, int count, int p, const double* var, double* pw, double* mono,
                                 int ld, int npt) {
  const int P1 = p + 1;
  for (int i = threadIdx.x; i < npt * (NS + 1); i += blockDim.x) {
    const int pt = i / (NS + 1), v = i % (NS + 1);
    const double x = var[pt * (NS + 1) + v];
    double* o = pw + (pt * (NS + 1) + v) * P1;
    double a = 1.0;
    for (int e = 0; e < P1; ++e) {
      o[e] = a;
      a *= x;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < npt * count; i += blockDim.x) {
    const int m = i / npt, pt = i % npt;
    const int* ex = T.expo + m * (NS + 1);
    const double* w = pw + pt * (NS + 1) * P1;
    double val = w[ex[0]];
#pragma unroll
    for (int v = 1; v <= NS; ++v) val *= w[v * P1 + ex[v]];
    mono[m * ld + pt] = val;
  }
}

// vhat = dUhat/dth, sigmahat = -grad Uhat (f[0..NS]) and optionally Uhat of
// basis function j+1 at point pt, one pass over the terms of Uhat.
template <int NS, bool WITH_U>
__device__ inline void eval_j(const Tab& T, int j, const double* mono, int ld, int pt, double* f, double* u) {
  double acc[NS + 2];
#pragma unroll
  for (int s = 0; s < NS + 2; ++s) acc[s] = 0.0;
  const int e1 = T.ue_ptr[j + 1];
  for (int e = T.ue_ptr[j]; e < e1; ++e) {
    const int* ix = T.ue_idx + e * (NS + 2);
    const double* cf = T.ue_coef + e * (NS + 2);
#pragma unroll
    for (int s = WITH_U ? 0 : 1; s < NS + 2; ++s) acc[s] += cf[s] * mono[ix[s] * ld + pt];
  }
#pragma unroll
  for (int s = 0; s <= NS; ++s) f[s] = acc[1 + s];
  if (WITH_U) *u = acc[0];
}

__device__ inline double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// LU without row exchanges of the augmented S x (S+1) matrix (S <= SMAX <= 64)
// by one wave, rows in registers: lane i holds row i; row k is broadcast with
// readlane.  The local matrices have a positive definite symmetric part
// (u^T A u = 1/2 B_top(u,u) + 1/2 B_bot(u,u) + penalty terms > 0 for Trefftz
// u, from eq. 4.1 and the divergence theorem), so every leading minor is
// nonzero and elimination with diagonal pivots is stable.  Returns false on a
// zero pivot.
template <int SMAX>
__device__ inline bool wave_lu_regs(const double* A, int lda, int S, double* x) {
  const int lane = threadIdx.x & 63;
  double r[SMAX + 1];
#pragma unroll
  for (int j = 0; j < SMAX; ++j) r[j] = (lane < S && j < S) ? A[lane * lda + j] : 0.0;
  r[SMAX] = lane < S ? A[lane * lda + S] : 0.0;
  bool ok = true;
#pragma unroll
  for (int k = 0; k < SMAX; ++k) {
    if (k < S) {
      const double pk = readlane_d(r[k], k);
      if (pk == 0.0) ok = false;
      const double l = lane > k ? r[k] / pk : 0.0;
#pragma unroll
      for (int j = k + 1; j <= SMAX; ++j)
        if (j < S || j == SMAX) r[j] -= l * readlane_d(r[j], k);
    }
  }
  if (!ok) return false;
#pragma unroll
  for (int k = SMAX - 1; k >= 0; --k) {
    if (k < S) {
      const double xk = readlane_d(r[SMAX], k) / readlane_d(r[k], k);
      if (lane == 0) x[k] = xk;
      if (lane < k) r[SMAX] -= r[k] * xk;
    }
  }
  return true;
}

// In-place LU without row exchanges of the S x S part of A (the right-hand
// side column is left alone): unit L below the diagonal, U on and above.
// Valid for the local matrices (positive definite symmetric part, see
// wave_lu_regs).  Returns false on a zero pivot.
__device__ inline bool block_lu_factor(double* A, long long lda, int S) {
  const int tid = threadIdx.x;
  for (int k = 0; k < S; ++k) {
    const double piv = A[k * lda + k];
    if (piv == 0.0) return false;
    for (int i = k + 1 + tid / 4; i < S; i += blockDim.x / 4) {
      const double l = A[i * lda + k] / piv;
      for (int j = k + 1 + (tid & 3); j < S; j += 4) A[i * lda + j] -= l * A[k * lda + j];
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < S; i += blockDim.x) A[i * lda + k] /= piv;
    __syncthreads();
  }
  return true;
}

// Solves L U x = b with the factors of block_lu_factor; b (LDS) is overwritten by x.
__device__ inline void block_lu_apply(const double* A, long long lda, int S, double* b) {
  const int tid = threadIdx.x;
  for (int k = 0; k < S; ++k) {
    const double bk = b[k];
    for (int i = k + 1 + tid; i < S; i += blockDim.x) b[i] -= A[i * lda + k] * bk;
    __syncthreads();
  }
  for (int k = S - 1; k >= 0; --k) {
    const double xk = b[k] / A[k * lda + k];
    __syncthreads();
    if (tid == 0) b[k] = xk;
    for (int i = tid; i < k; i += blockDim.x) b[i] -= A[i * lda + k] * xk;
    __syncthreads();
  }
}

// Workgroup LU with partial pivoting of the augmented S x (S+1) matrix
// (LDS or global memory).  s_piv: shared scratch.  Returns false on a zero pivot.
__device__ inline bool block_lu_solve(double* A, long long lda, int S, double* x, int* s_piv) {
  const int tid = threadIdx.x;
  for (int k = 0; k < S; ++k) {
    if (tid < 64) {
      double best = -1.0;
      int bi = S;
      for (int r = k + tid; r < S; r += 64) {
        const double v = fabs(A[r * lda + k]);
        if (v > best) {
          best = v;
          bi = r;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (tid == 0) *s_piv = bi < S ? bi : k;  // (a column of NaNs keeps its row)
    }
    __syncthreads();
    const int pr = *s_piv;
    if (pr != k)
      for (int j = k + tid; j <= S; j += blockDim.x) {
        const double t = A[k * lda + j];
        A[k * lda + j] = A[pr * lda + j];
        A[pr * lda + j] = t;
      }
    __syncthreads();
    const double piv = A[k * lda + k];
    if (piv == 0.0) return false;
    // four threads per row: multiplier, then the row update (the multiplier
    // column k is written only after the barrier below)
    for (int i = k + 1 + tid / 4; i < S; i += blockDim.x / 4) {
      const double l = A[i * lda + k] / piv;
      for (int j = k + 1 + (tid & 3); j <= S; j += 4) A[i * lda + j] -= l * A[k * lda + j];
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < S; i += blockDim.x) A[i * lda + k] /= piv;
    __syncthreads();
  }
  for (int k = S - 1; k >= 0; --k) {
    const double xk = A[k * lda + S] / A[k * lda + k];
    if (tid == 0) x[k] = xk;
    for (int i = tid; i < k; i += blockDim.x) A[i * lda + S] -= A[i * lda + k] * xk;
    __syncthreads();
  }
  return true;
}

// Blocked LU with partial pivoting of the augmented S x (S+1) matrix in global
// memory (the workgroup's slot), then back substitution into x (LDS).  The
// pivot rule is that of block_lu_solve (largest magnitude in the pivot column,
// ties to the lower row); the elimination is organised in panels of nb columns
// so that the trailing matrix is read and written once per panel rather than
// once per column:
//   1. rows k0..S-1 of the panel's columns are copied to LDS (column-major) and
//      factored there: pivot search, exchange of whole panel rows, multipliers,
//      rank-1 update of the panel's remaining columns;
//   2. for each column right of the panel (the right-hand side included) one
//      thread applies the panel's row exchanges and solves L11 u = a for the
//      panel's rows: U12, kept in LDS and written back;
//   3. A22 -= L21 U12 on the FP64 matrix cores (16x16 tiles, 4 terms per step);
//   4. back substitution in blocks of nb rows from the bottom: one wave solves
//      the diagonal block with its rows in registers, then every thread
//      updates the right-hand sides of the rows above.
// The multipliers below the panel's rows are not written back: the right-hand
// side is carried as column S, and only U is read afterwards.  ws holds
// lu_ws_doubles(S, nb) doubles; nb is a multiple of 4, at most 32.  Returns
// false (for the whole workgroup) on a zero pivot.
__device__ inline bool panel_lu_solve(double* A, long long lda, int S, int nb, double* x, double* ws) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
  const int ldp = lu_ldp(S), ldu = lu_ldu(S);
  double* Pn = ws;                                            // panel: Pn[j * ldp + r], r = row - k0
  double* Ub = ws + (long long)nb * ldp;                      // U12: Ub[kk * ldu + c], column k0 + nbb + c
  int* orig = reinterpret_cast<int*>(Ub + (long long)nb * ldu);  // orig[r]: old panel row now at position r
  int* piv = orig + S;                                        // piv[kk]: position exchanged with kk
  for (int k0 = 0; k0 < S; k0 += nb) {
    const int nbb = min(nb, S - k0), R = S - k0;
    // (loads batched ahead of the LDS stores)
    for (int i0 = tid; i0 < R * nbb; i0 += 8 * blockDim.x) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + u * blockDim.x, r = i / nbb, j = i - r * nbb;
        v[u] = i < R * nbb ? A[(long long)(k0 + r) * lda + k0 + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + u * blockDim.x, r = i / nbb, j = i - r * nbb;
        if (i < R * nbb) Pn[j * ldp + r] = v[u];
      }
    }
    for (int r = tid; r < R; r += blockDim.x) orig[r] = r;
    __syncthreads();
    for (int kk = 0; kk < nbb; ++kk) {
      if (wave == 0) {
        double best = -1.0;
        int bi = R;
        for (int r = kk + lane; r < R; r += 64) {
          const double v = fabs(Pn[kk * ldp + r]);
          if (v > best) {
            best = v;
            bi = r;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          const double ob = __shfl_xor(best, off, 64);
          const int oi = __shfl_xor(bi, off, 64);
          if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
          }
        }
        if (lane == 0) piv[kk] = bi < R ? bi : kk;  // (a column of NaNs keeps its row)
      }
      __syncthreads();
      const int pr = piv[kk];
      if (pr != kk) {
        for (int j = tid; j < nbb; j += blockDim.x) {
          const double t = Pn[j * ldp + kk];
          Pn[j * ldp + kk] = Pn[j * ldp + pr];
          Pn[j * ldp + pr] = t;
        }
        if (tid == 0) {
          const int t = orig[kk];
          orig[kk] = orig[pr];
          orig[pr] = t;
        }
      }
      __syncthreads();
      const double pv = Pn[kk * ldp + kk];
      if (pv == 0.0) return false;
      // one thread per row below the pivot: its multiplier, then its panel row
      for (int r = kk + 1 + tid; r < R; r += blockDim.x) {
        const double l = Pn[kk * ldp + r] / pv;
        Pn[kk * ldp + r] = l;
        for (int j = kk + 1; j < nbb; ++j) Pn[j * ldp + r] -= l * Pn[j * ldp + kk];
      }
      __syncthreads();
    }
    // U11 back to global memory (the diagonal block of the back substitution)
    for (int i = tid; i < nbb * nbb; i += blockDim.x) {
      const int r = i / nbb, j = i - r * nbb;
      if (j >= r) A[(long long)(k0 + r) * lda + k0 + j] = Pn[j * ldp + r];
    }
    // U12, one thread per column: the exchanged column's entries at positions
    // kk < nbb come from rows orig[kk]; the rows displaced below them (positions
    // piv[kk] >= nbb) get entries of rows < nbb, which are overwritten only at
    // the end, after every load of this column
    const int r0 = k0 + nbb, W = S + 1 - r0;
    for (int c = tid; c < W; c += blockDim.x) {
      const long long col = r0 + c;
      double v[32];
#pragma unroll
      for (int kk = 0; kk < 32; ++kk) v[kk] = kk < nbb ? A[(long long)(k0 + orig[kk]) * lda + col] : 0.0;
#pragma unroll
      for (int kk = 0; kk < 32; ++kk)
        if (kk < nbb) Ub[kk * ldu + c] = v[kk];
      for (int kk = 0; kk < nbb; ++kk) {
        const int pos = piv[kk];
        if (pos >= nbb) A[(long long)(k0 + pos) * lda + col] = A[(long long)(k0 + orig[pos]) * lda + col];
      }
      for (int kk = 0; kk < nbb; ++kk) {
        double u = Ub[kk * ldu + c];
        for (int m = 0; m < kk; ++m) u -= Pn[m * ldp + kk] * Ub[m * ldu + c];
        Ub[kk * ldu + c] = u;
        A[(long long)(k0 + kk) * lda + col] = u;
      }
    }
    __syncthreads();
    // A22 -= L21 U12: tile (ti, tj) covers rows r0 + 16 ti.., columns r0 + 16 tj..;
    // lane l supplies L21[row l%16][k l/16] and U12[k l/16][column l%16], and
    // element e of the result is row l/16 + 4e, column l%16
    // (four tiles per wave at a time, their loads issued together)
    const int nr = S - r0;
    const int tr = (nr + 15) / 16, tc = (W + 15) / 16, nt = tr * tc;
    for (int tb = wave * 4; tb < nt; tb += nwave * 4) {
      d4 acc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = min(tb + u, nt - 1);
        const int i0 = r0 + (t / tc) * 16, jc = r0 + (t % tc) * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = i0 + (lane >> 4) + 4 * e;
          acc[u][e] = (i < S && jc <= S) ? A[(long long)i * lda + jc] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = min(tb + u, nt - 1);
        const int ia = r0 + (t / tc) * 16 + (lane & 15), jc = r0 + (t % tc) * 16 + (lane & 15);
        for (int kq = 0; kq < nbb; kq += 4) {
          const int kk = kq + (lane >> 4);
          const double a = (ia < S && kk < nbb) ? -Pn[kk * ldp + (ia - k0)] : 0.0;
          const double b = (jc <= S && kk < nbb) ? Ub[kk * ldu + (jc - r0)] : 0.0;
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (tb + u < nt) {
          const int t = tb + u;
          const int i0 = r0 + (t / tc) * 16, jc = r0 + (t % tc) * 16 + (lane & 15);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int i = i0 + (lane >> 4) + 4 * e;
            if (i < S && jc <= S) A[(long long)i * lda + jc] = acc[u][e];
          }
        }
      }
    }
    __syncthreads();
  }
  // back substitution
  for (int i = tid; i < S; i += blockDim.x) x[i] = A[(long long)i * lda + S];
  __syncthreads();
  for (int kb = ((S - 1) / nb) * nb; kb >= 0; kb -= nb) {
    const int nbb = min(nb, S - kb);
    if (wave == 0) {
      double r[32];
#pragma unroll
      for (int j = 0; j < 32; ++j) r[j] = (lane < nbb && j < nbb) ? A[(long long)(kb + lane) * lda + kb + j] : 0.0;
      double bi = lane < nbb ? x[kb + lane] : 0.0;
#pragma unroll
      for (int k = 31; k >= 0; --k) {
        if (k < nbb) {
          const double xk = readlane_d(bi, k) / readlane_d(r[k], k);
          if (lane < k) bi -= r[k] * xk;
          if (lane == k) bi = xk;
        }
      }
      if (lane < nbb) x[kb + lane] = bi;
    }
    __syncthreads();
    for (int i = tid; i < kb; i += blockDim.x) {
      const double* row = A + (long long)i * lda + kb;
      double v[32];
#pragma unroll
      for (int j = 0; j < 32; ++j) v[j] = j < nbb ? row[j] : 0.0;
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < 32; ++j)
        if (j < nbb) s += v[j] * x[kb + j];
      x[i] -= s;
    }
    __syncthreads();
  }
  return true;
}

}  // namespace

// Solves one tent; called by every thread of the workgroup.  All early returns
// are taken by the whole workgroup (their conditions are workgroup-uniform).

// Gram block (r, r) of a tent from the moments NU (moment mode), NZ test
// functions i = i0 .. i0+NZ-1 at a time:  Z_i[b][l] = sum over the terms
// (a, k, al) of function i of al H_ab(k, l) (one thread per (i, l)), then
// A_ij += sum over the terms (b, l, be) of function j of be Z_i[b][l] (one
// thread per j, the table terms of j loaded once for the NZ rows).  Top Gram
// (dirichlet = false): H_00 = H_dd = nu, H_0d = H_d0 = -c nu_d (lower triangle
// computed, mirrored).  Dirichlet faces (dirichlet = true): H_00 = alpha c^2 nu,
// H_0d = c nu_d (row v, column sigma_d), all j.  Every sum keeps the term order
// of the table, so the result does not depend on NZ.
template <int NS, int NZ>
__device__ inline void moment_gram_pass(const int* fo_ptr, const int* fo_idx, const double* fo_coef,
                                        const int* K2, int M1, int M2, int NW, const double* NU, double* Z,
                                        double cr, double alpha, bool dirichlet, double* A, long long lda,
                                        int row0) {
  const int tid = threadIdx.x;
  const double ca = alpha * cr * cr;
  for (int i0 = 0; i0 < NW; i0 += NZ) {
    const int nzi = min(NZ, NW - i0);
    // Z of the functions i0 + q: item q M1 + l, its sums in registers over all
    // table terms of the function (in term order); terms in groups of four with
    // their product-index loads (global) issued together, a missing term entering
    // with coefficient 0 at index 0
    for (int it = tid; it < nzi * M1; it += blockDim.x) {
      const int q = it / M1, l = it - q * M1, i = i0 + q;
      double z[NS + 1];
#pragma unroll
      for (int c = 0; c <= NS; ++c) z[c] = 0.0;
      const int amax = dirichlet ? 0 : NS;
      for (int a = 0; a <= amax; ++a) {
        const int row = i * (NS + 1) + a;
        const int e1 = fo_ptr[row + 1];
        for (int e = fo_ptr[row]; e < e1; e += 4) {
          int kk[4];
          double al[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            kk[u] = e + u < e1 ? fo_idx[e + u] : 0;
            al[u] = e + u < e1 ? fo_coef[e + u] : 0.0;
          }
          int b2[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) b2[u] = K2[kk[u] * M1 + l];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int b = b2[u];
            if (dirichlet) {
              z[0] += ca * al[u] * NU[b];
#pragma unroll
              for (int d = 0; d < NS; ++d) z[1 + d] += cr * al[u] * NU[(1 + d) * M2 + b];
            } else if (a == 0) {
              z[0] += al[u] * NU[b];
#pragma unroll
              for (int d = 0; d < NS; ++d) z[1 + d] -= cr * al[u] * NU[(1 + d) * M2 + b];
            } else {
#pragma unroll
              for (int c = 1; c <= NS; ++c)
                if (c == a) z[c] += al[u] * NU[b];
              z[0] -= cr * al[u] * NU[a * M2 + b];
            }
          }
        }
      }
#pragma unroll
      for (int c = 0; c <= NS; ++c) Z[(q * (NS + 1) + c) * M1 + l] = z[c];
    }
    __syncthreads();
    const int jmax = dirichlet ? NW - 1 : i0 + nzi - 1;
    for (int j = tid; j <= jmax; j += blockDim.x) {
      // the terms of function j (components b = 0..NS, consecutive in the table)
      // eight at a time: their table loads are issued together; each row's sum
      // keeps the term order (rows q >= nzi read words of no function and are
      // not stored)
      int bnd[NS + 2];
#pragma unroll
      for (int b = 0; b <= NS + 1; ++b) bnd[b] = fo_ptr[j * (NS + 1) + b];
      double acc[NZ];
#pragma unroll
      for (int q = 0; q < NZ; ++q) acc[q] = 0.0;
      for (int e = bnd[0]; e < bnd[NS + 1]; e += 8) {
        int ix[8];
        double cf[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          ix[u] = e + u < bnd[NS + 1] ? fo_idx[e + u] : 0;
          cf[u] = e + u < bnd[NS + 1] ? fo_coef[e + u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          int b = 0;
#pragma unroll
          for (int c = 1; c <= NS; ++c) b += e + u >= bnd[c] ? 1 : 0;
          if (e + u < bnd[NS + 1])
#pragma unroll
            for (int q = 0; q < NZ; ++q) acc[q] += cf[u] * Z[(q * (NS + 1) + b) * M1 + ix[u]];
        }
      }
#pragma unroll
      for (int q = 0; q < NZ; ++q) {
        const int i = i0 + q;
        if (q < nzi && (dirichlet || j <= i)) {
          A[(long long)(row0 + i) * lda + row0 + j] += acc[q];
          if (!dirichlet && j != i) A[(long long)(row0 + j) * lda + row0 + i] += acc[q];
        }
      }
    }
    __syncthreads();
  }
}

// The Gram block with as many test functions per pass (1, 2, 4 or 8) as the
// Z rows fit in zcap doubles at Z.
template <int NS>
__device__ inline void moment_gram_block(const int* fo_ptr, const int* fo_idx, const double* fo_coef,
                                         const int* K2, int M1, int M2, int NW, const double* NU, double* Z,
                                         long long zcap, double cr, double alpha, bool dirichlet, double* A,
                                         long long lda, int row0) {
  const long long per = (long long)(NS + 1) * M1;
  if (zcap >= 8 * per)
    moment_gram_pass<NS, 8>(fo_ptr, fo_idx, fo_coef, K2, M1, M2, NW, NU, Z, cr, alpha, dirichlet, A, lda, row0);
  else if (zcap >= 4 * per)
    moment_gram_pass<NS, 4>(fo_ptr, fo_idx, fo_coef, K2, M1, M2, NW, NU, Z, cr, alpha, dirichlet, A, lda, row0);
  else if (zcap >= 2 * per)
    moment_gram_pass<NS, 2>(fo_ptr, fo_idx, fo_coef, K2, M1, M2, NW, NU, Z, cr, alpha, dirichlet, A, lda, row0);
  else
    moment_gram_pass<NS, 1>(fo_ptr, fo_idx, fo_coef, K2, M1, M2, NW, NU, Z, cr, alpha, dirichlet, A, lda, row0);
}


// Moments over the points of one speed group (moment mode): top moments of the
// monomials of degree <= 2p-2 weighted by w and w g_d (NU), bottom moments of the
// monomials of degree <= p weighted by w (BU) and by the incoming-data terms of
// the right-hand side (BV), and the weight and U sums of the recovery row.

// Moment tasks of this thread (t = tid + s * blockDim.x), packed words in registers.
template <int NSLOT>
struct TaskRegs {
  unsigned w0[NSLOT], w1[NSLOT], w2[NSLOT];
};
// slot s of a thread holds task t0 + s * stride (by default the thread index
// and the block size)
template <int NSLOT>
__device__ inline void load_tasks(const int* task, int ntask, TaskRegs<NSLOT>& R, int t0 = -1, int stride = 0) {
  if (t0 < 0) t0 = threadIdx.x;
  if (stride <= 0) stride = blockDim.x;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int t = t0 + s * stride;
    R.w0[s] = t < ntask ? (unsigned)task[t * kTaskInts] : 0u;
    R.w1[s] = t < ntask ? (unsigned)task[t * kTaskInts + 1] : 0xFFFFFFFFu;
    R.w2[s] = t < ntask ? (unsigned)task[t * kTaskInts + 2] : 0xFFFFFFFFu;
  }
}
__device__ inline int task_exp(unsigned w0, int v) { return (int)((w0 >> (5 * v)) & 31u); }
template <int NSLOT>
__device__ inline int task_idx(const TaskRegs<NSLOT>& R, int s, int c) {
  const unsigned w = c < 2 ? R.w1[s] : R.w2[s];
  const unsigned i = (c & 1) ? (w >> 16) : (w & 0xFFFFu);
  return i == 0xFFFFu ? -1 : (int)i;
}

template <int NS>
__device__ inline void moment_points(const double* lam_ref, const double* w_ref, const double* state, int Q,
                                           const double* EL, int ELS, const int* gel, int npts, const double* XV,
                                           double cr, double hr, double tmid, double dt, int p, int PCH, int M1,
                                           int M2, int Mm, const int* task1, int ntask1, const int* task2,
                                           int ntask2, double* NU, double* BV,
                                           double* BU, double* PV, double* PW, double* PD, double* PG, double* POWT,
                                           double* POWB, double* A00r, double* r0r) {
  const int tid = threadIdx.x;
  const int E2 = 2 * p - 1;
  const double ic2 = 1.0 / (cr * cr);
  for (int i = tid; i < (NS + 1) * M2 + (NS + 1) * M1 + Mm; i += blockDim.x) NU[i] = 0.0;
  double sw_acc = 0.0, su_acc = 0.0;
  TaskRegs<kTaskSlots> RT;
  TaskRegs<kTaskSlots1> RB;
  load_tasks(task2, ntask2, RT);
  load_tasks(task1, ntask1, RB);
  __syncthreads();
  for (int f0 = 0; f0 < npts; f0 += PCH) {
    const int nc = min(PCH, npts - f0);
    for (int pt = tid; pt < nc; pt += blockDim.x) {
      const int f = f0 + pt;
      const int li = gel[f / Q];
      const int q = f % Q;
      const double* R = EL + li * ELS;
      const int lV = (int)R[El<NS>::LV];
      const int e = (int)R[El<NS>::E];
      const double* lam = lam_ref + (size_t)q * (NS + 1);
      double xt[NS], pho = 0.0;
      for (int d = 0; d < NS; ++d) xt[d] = 0.0;
      for (int k = 0; k <= NS; ++k) {
        pho += lam[k] * R[El<NS>::TAU + k];
        for (int d = 0; d < NS; ++d) xt[d] += lam[k] * R[El<NS>::X + k * NS + d];
      }
      const double phi = pho + lam[lV] * dt;
      const double w = w_ref[q] * R[El<NS>::DET];
      const double* st = state + (size_t)e * (NS + 2) * Q;
      const double vb = st[q];
      double sg = 0.0;
      for (int d = 0; d < NS; ++d) sg += st[(1 + d) * Q + q] * R[El<NS>::GOLD + d];
      PD[pt * (NS + 2)] = w * (ic2 * vb - sg);
      for (int d = 0; d < NS; ++d) PD[pt * (NS + 2) + 1 + d] = w * (st[(1 + d) * Q + q] - vb * R[El<NS>::GOLD + d]);
      PD[pt * (NS + 2) + NS + 1] = w * st[(NS + 1) * Q + q];
      PV[pt * (NS + 1)] = cr * (phi - tmid) / hr;
      PV[(PCH + pt) * (NS + 1)] = cr * (pho - tmid) / hr;
      for (int d = 0; d < NS; ++d) {
        const double xh = (xt[d] - XV[d]) / hr;
        PV[pt * (NS + 1) + 1 + d] = xh;
        PV[(PCH + pt) * (NS + 1) + 1 + d] = xh;
        PG[pt * NS + d] = w * R[El<NS>::GNEW + d];
      }
      PW[pt] = w;
      sw_acc += w;
      su_acc += PD[pt * (NS + 2) + NS + 1];
    }
    __syncthreads();
    for (int i = tid; i < nc * (NS + 1); i += blockDim.x) {
      const int pt = i / (NS + 1), v = i % (NS + 1);
      double x = PV[pt * (NS + 1) + v], a = 1.0;
      double* o = POWT + (pt * (NS + 1) + v) * E2;
      for (int ee = 0; ee < E2; ++ee) {
        o[ee] = a;
        a *= x;
      }
      x = PV[(PCH + pt) * (NS + 1) + v];
      a = 1.0;
      o = POWB + (pt * (NS + 1) + v) * (p + 1);
      for (int ee = 0; ee <= p; ++ee) {
        o[ee] = a;
        a *= x;
      }
    }
    __syncthreads();
    // top moments, one task (a run of up to 4 monomials that differ in the last
    // exponent only) per slot: the shared prefix is formed once per point
#pragma unroll
    for (int sl = 0; sl < kTaskSlots; ++sl) {
      if (tid + sl * (int)blockDim.x >= ntask2) break;
      const unsigned w0 = RT.w0[sl];
      int e[NS];
#pragma unroll
      for (int v = 0; v < NS; ++v) e[v] = task_exp(w0, v);
      const int d0 = task_exp(w0, 3);
      double a0[4], ad[4][NS];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        a0[c] = 0.0;
#pragma unroll
        for (int d = 0; d < NS; ++d) ad[c][d] = 0.0;
      }
#pragma unroll 1
      for (int pt = 0; pt < nc; ++pt) {
        const double* pw = POWT + pt * (NS + 1) * E2;
        double pre = pw[e[0]];
#pragma unroll
        for (int v = 1; v < NS; ++v) pre *= pw[v * E2 + e[v]];
        const double z = E2 > 1 ? pw[NS * E2 + 1] : 0.0;
        double mv = pre * pw[NS * E2 + d0];
        const double w = PW[pt];
        double wg[NS];
#pragma unroll
        for (int d = 0; d < NS; ++d) wg[d] = PG[pt * NS + d];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          a0[c] += w * mv;
#pragma unroll
          for (int d = 0; d < NS; ++d) ad[c][d] += wg[d] * mv;
          mv *= z;
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int b = task_idx(RT, sl, c);
        if (b < 0) continue;
        NU[b] += a0[c];
#pragma unroll
        for (int d = 0; d < NS; ++d) NU[(1 + d) * M2 + b] += ad[c][d];
      }
    }
    // bottom moments (monomials of degree <= p), same task scheme
#pragma unroll
    for (int sl = 0; sl < kTaskSlots1; ++sl) {
      if (tid + sl * (int)blockDim.x >= ntask1) break;
      const unsigned w0 = RB.w0[sl];
      int e[NS];
#pragma unroll
      for (int v = 0; v < NS; ++v) e[v] = task_exp(w0, v);
      const int d0 = task_exp(w0, 3);
      double bu[4], bv[4][NS + 1];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        bu[c] = 0.0;
#pragma unroll
        for (int q = 0; q <= NS; ++q) bv[c][q] = 0.0;
      }
#pragma unroll 1
      for (int pt = 0; pt < nc; ++pt) {
        const double* pw = POWB + pt * (NS + 1) * (p + 1);
        double pre = pw[e[0]];
#pragma unroll
        for (int v = 1; v < NS; ++v) pre *= pw[v * (p + 1) + e[v]];
        const double z = pw[NS * (p + 1) + 1];
        double mv = pre * pw[NS * (p + 1) + d0];
        const double w = PW[pt];
        double dd[NS + 1];
#pragma unroll
        for (int q = 0; q <= NS; ++q) dd[q] = PD[pt * (NS + 2) + q];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          bu[c] += w * mv;
#pragma unroll
          for (int q = 0; q <= NS; ++q) bv[c][q] += dd[q] * mv;
          mv *= z;
        }
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k = task_idx(RB, sl, c);
        if (k < 0) continue;
        BU[k] += bu[c];
        if (k < M1)
#pragma unroll
          for (int q = 0; q <= NS; ++q) BV[q * M1 + k] += bv[c][q];
      }
    }
    __syncthreads();
  }
  // the recovery row's weight and U sums: each set-up thread's, then the block's
  block_sum2(sw_acc, su_acc, PW);
  if (tid == 0) {
    *A00r += sw_acc;
    *r0r += su_acc;
  }
}


// Moments over the points of one speed group (3+1D), element by element, with
// the top moments on the FP64 matrix cores.  A moment monomial factors as
// m_b = L_i(th, xh_1) R_j(xh_2, xh_3); over the points of one element the
// moments of all products are the tiles of C_e = (w L)^T R, a 16x16x4 MFMA
// per tile and four points (lane l: row or column l%16, point l/16 of the
// step).  grad phi_new is constant on an element, so after its last chunk
//   nu[b] += C_e[b],  nu_d[b] += g_d C_e[b]   (b = mt_map of the tile entry)
// and the tiles restart from zero.  The bottom moments and the recovery-row
// sums are those of moment_points (VALU tasks); with at most 64 (128) tasks the
// tasks are repeated in 4 (2) groups of waves, group s taking the points
// s, s + nsplit, ... of every chunk, so that all waves share them.  The first
// task slot of a thread sums over all chunks in registers; the groups add
// their sums in group order after the last chunk.  Chunks hold at most PCH
// points of one element (PCH a multiple of 4: every k-step reads inside the
// chunk's regions; points past the chunk enter with zero operands).
template <int NS>
__device__ inline void moment_points_mt(const double* lam_ref, const double* w_ref, const double* state, int Q,
                                        const double* EL, int ELS, const int* gel, int nel, const double* XV,
                                        double cr, double hr, double tmid, double dt, int p, int PCH, int M1, int M2,
                                        int Mm, const int* task1, int ntask1, int ntile, const int* mt_ex,
                                        const int* mt_map, double* NU, double* BV, double* BU, double* PV, double* PW,
                                        double* PD, double* POWT, double* POWB, double* A00r, double* r0r) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: slot tests are scalar branches
  const int E2 = 2 * p - 1;
  const double ic2 = 1.0 / (cr * cr);
  for (int i = tid; i < (NS + 1) * M2 + (NS + 1) * M1 + Mm; i += blockDim.x) NU[i] = 0.0;
  const int nslot0 = (ntile + 3) >> 2;  // slots of wave 0 (the most): tiles wave + 4 s
  double sw_acc = 0.0, su_acc = 0.0;
  // bottom tasks: groups of waves (every task of the group in one slot when
  // nsplit > 1, so the groups never write a moment word in the same pass)
  const int nwt = max(1, (ntask1 + 63) >> 6);
  const int nsplit = (blockDim.x == 256 && nwt <= 2) ? 4 / nwt : 1;
  const int span = blockDim.x / nsplit, split = tid / span, ttask = tid - split * span;
  TaskRegs<kTaskSlots1> RB;
  load_tasks(task1, ntask1, RB, ttask, span);
  double bu0[4], bv0[4][NS + 1];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    bu0[c] = 0.0;
#pragma unroll
    for (int q = 0; q <= NS; ++q) bv0[c][q] = 0.0;
  }
  // sums of the task in slot sl over the points split, split + nsplit, ... < nc;
  // the LDS words of the next point are loaded before the current point's
  // products (the last point loads itself again)
  auto bottom_sums = [&](int sl, int nc, double (&bu)[4], double (&bv)[4][NS + 1]) {
    const unsigned w0 = RB.w0[sl];
    int e[NS];
#pragma unroll
    for (int v = 0; v < NS; ++v) e[v] = task_exp(w0, v);
    const int d0 = task_exp(w0, 3);
    if (split >= nc) return;
    double f[NS + 1], z, w, dd[NS + 1];
    auto load = [&](int pt, double (&f_)[NS + 1], double& z_, double& w_, double (&dd_)[NS + 1]) {
      const double* pw = POWB + pt * (NS + 1) * (p + 1);
#pragma unroll
      for (int v = 0; v < NS; ++v) f_[v] = pw[v * (p + 1) + e[v]];
      f_[NS] = pw[NS * (p + 1) + d0];
      z_ = pw[NS * (p + 1) + 1];
      w_ = PW[pt];
#pragma unroll
      for (int q = 0; q <= NS; ++q) dd_[q] = PD[pt * (NS + 2) + q];
    };
    load(split, f, z, w, dd);
    for (int pt = split; pt < nc; pt += nsplit) {
      double fn[NS + 1], zn, wn, ddn[NS + 1];
      load(min(pt + nsplit, nc - 1), fn, zn, wn, ddn);
      double mv = f[0];
#pragma unroll
      for (int v = 1; v <= NS; ++v) mv *= f[v];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        bu[c] += w * mv;
#pragma unroll
        for (int q = 0; q <= NS; ++q) bv[c][q] += dd[q] * mv;
        mv *= z;
      }
#pragma unroll
      for (int v = 0; v <= NS; ++v) f[v] = fn[v];
      z = zn;
      w = wn;
#pragma unroll
      for (int q = 0; q <= NS; ++q) dd[q] = ddn[q];
    }
  };
  // slot 0: exponents of the task's prefix and run start, and the sums of one point
  int e0x[NS], d0x;
#pragma unroll
  for (int v = 0; v < NS; ++v) e0x[v] = task_exp(RB.w0[0], v);
  d0x = task_exp(RB.w0[0], 3);
  auto bottom_point0 = [&](int pt) {
    const double* pw = POWB + pt * (NS + 1) * (p + 1);
    double mv = pw[e0x[0]];
#pragma unroll
    for (int v = 1; v < NS; ++v) mv *= pw[v * (p + 1) + e0x[v]];
    mv *= pw[NS * (p + 1) + d0x];
    const double z = pw[NS * (p + 1) + 1];
    const double w = PW[pt];
    double dd[NS + 1];
#pragma unroll
    for (int q = 0; q <= NS; ++q) dd[q] = PD[pt * (NS + 2) + q];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      bu0[c] += w * mv;
#pragma unroll
      for (int q = 0; q <= NS; ++q) bv0[c][q] += dd[q] * mv;
      mv *= z;
    }
  };
  auto bottom_flush = [&](int sl, const double (&bu)[4], const double (&bv)[4][NS + 1]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int k = task_idx(RB, sl, c);
      if (k < 0) continue;
      BU[k] += bu[c];
      if (k < M1)
#pragma unroll
        for (int q = 0; q <= NS; ++q) BV[q * M1 + k] += bv[c][q];
    }
  };
  unsigned tex[kMomTileSlots];
  d4 acc[kMomTileSlots];
#pragma unroll
  for (int s = 0; s < kMomTileSlots; ++s) {
    const int t = wave + 4 * s;
    tex[s] = t < ntile ? (unsigned)mt_ex[t * 16 + (lane & 15)] : 0u;
    acc[s] = d4{0.0, 0.0, 0.0, 0.0};
  }
  __syncthreads();
  // chunks of at most PCH points of one element, flattened: chunk c covers
  // element gel[c / cpe], points (c % cpe) PCH .. ; thread pt < PCH keeps the
  // global data of its point of the next chunk in registers (state, reference
  // coordinates, weight), loaded while the current chunk is processed
  const int cpe = (Q + PCH - 1) / PCH;
  const int nchunk = nel * cpe;
  double g_st[NS + 2], g_lam[NS + 1], g_w = 0.0;
  auto fetch = [&](int c) {
    const int pt = tid;
    if (c < nchunk && pt < PCH) {
      const int q = (c % cpe) * PCH + pt;
      if (q < Q) {
        const double* Rn = EL + gel[c / cpe] * ELS;
        const double* st = state + (size_t)(int)Rn[El<NS>::E] * (NS + 2) * Q;
#pragma unroll
        for (int k = 0; k < NS + 2; ++k) g_st[k] = gload(st + k * Q + q);
#pragma unroll
        for (int k = 0; k <= NS; ++k) g_lam[k] = gload(lam_ref + (size_t)q * (NS + 1) + k);
        g_w = gload(w_ref + q);
      }
    }
  };
  fetch(0);
  for (int cc = 0; cc < nchunk; ++cc) {
    const int ei = cc / cpe, q0 = (cc % cpe) * PCH;
    const double* R = EL + gel[ei] * ELS;
    {
      const int nc = min(PCH, Q - q0), nc4 = (nc + 3) & ~3;
      if (tid < nc) {
        const int pt = tid;
        const int lV = (int)R[El<NS>::LV];
        double xt[NS], pho = 0.0;
        for (int d = 0; d < NS; ++d) xt[d] = 0.0;
        for (int k = 0; k <= NS; ++k) {
          pho += g_lam[k] * R[El<NS>::TAU + k];
          for (int d = 0; d < NS; ++d) xt[d] += g_lam[k] * R[El<NS>::X + k * NS + d];
        }
        const double phi = pho + g_lam[lV] * dt;
        const double w = g_w * R[El<NS>::DET];
        const double vb = g_st[0];
        double sg = 0.0;
        for (int d = 0; d < NS; ++d) sg += g_st[1 + d] * R[El<NS>::GOLD + d];
        PD[pt * (NS + 2)] = w * (ic2 * vb - sg);
        for (int d = 0; d < NS; ++d) PD[pt * (NS + 2) + 1 + d] = w * (g_st[1 + d] - vb * R[El<NS>::GOLD + d]);
        PD[pt * (NS + 2) + NS + 1] = w * g_st[NS + 1];
        PV[pt * (NS + 1)] = cr * (phi - tmid) / hr;
        PV[(PCH + pt) * (NS + 1)] = cr * (pho - tmid) / hr;
        for (int d = 0; d < NS; ++d) {
          const double xh = (xt[d] - XV[d]) / hr;
          PV[pt * (NS + 1) + 1 + d] = xh;
          PV[(PCH + pt) * (NS + 1) + 1 + d] = xh;
        }
        PW[pt] = w;
        sw_acc += w;
        su_acc += w * g_st[NS + 1];
      } else if (tid < nc4) {
        // points past the chunk up to the next multiple of 4: weight 0 and zero
        // coordinates, so that the top tiles read finite powers and add nothing
        const int pt = tid;
        for (int v = 0; v <= NS; ++v) PV[pt * (NS + 1) + v] = 0.0;
        PW[pt] = 0.0;
      }
      __syncthreads();
      // powers of the top coordinates (those of th times the weight: the A
      // operand of the top tiles is w L) for nc4 points, of the bottom ones for nc
      for (int i = tid; i < nc4 * (NS + 1); i += blockDim.x) {
        const int pt = i / (NS + 1), v = i % (NS + 1);
        double x = PV[pt * (NS + 1) + v], a = v == 0 ? PW[pt] : 1.0;
        double* o = POWT + (pt * (NS + 1) + v) * E2;
        for (int ee = 0; ee < E2; ++ee) {
          o[ee] = a;
          a *= x;
        }
        if (pt >= nc) continue;
        x = PV[(PCH + pt) * (NS + 1) + v];
        a = 1.0;
        o = POWB + (pt * (NS + 1) + v) * (p + 1);
        for (int ee = 0; ee <= p; ++ee) {
          o[ee] = a;
          a *= x;
        }
      }
      __syncthreads();
      // the next chunk's global data, in flight during the moments of this chunk
      // (no barrier between here and the chunk's end)
      fetch(cc + 1);
      // top moment tiles of this chunk.  The operand loads of all slots are issued
      // together: every index lies in this point's power row (a slot past the
      // wave's tiles has exponents 0); the points past nc up to nc4 have weight 0
      // Every wave runs the slot count of wave 0 (a compile-time count, so no
      // branches in the loop): a slot past the wave's tiles accumulates finite
      // values that are never folded.
      const int nks = nc4 >> 2;
      // The power words of step ks + 1 are loaded before the products of step ks
      // (the last step loads itself again).  The bottom moments of slot 0 for the
      // step's points of this wave group (pt = 4 ks + split + j, j a multiple of
      // nsplit) run on the VALU between the step's matrix-core instructions,
      // which execute meanwhile; every group takes its points in ascending order.
      const bool bot0 = ttask < ntask1;
      auto top_tiles = [&](auto nsl_c) {
        constexpr int NSL = decltype(nsl_c)::value;
        double f[NSL][4];
        auto load = [&](int ks, double (&f_)[NSL][4]) {
          const double* pw = POWT + (ks * 4 + (lane >> 4)) * (NS + 1) * E2;
#pragma unroll
          for (int s = 0; s < NSL; ++s) {
            const unsigned ex = tex[s];
            f_[s][0] = pw[ex & 31u];
            f_[s][1] = pw[E2 + ((ex >> 5) & 31u)];
            f_[s][2] = pw[2 * E2 + ((ex >> 10) & 31u)];
            f_[s][3] = pw[3 * E2 + ((ex >> 15) & 31u)];
          }
        };
        load(0, f);
        for (int ks = 0; ks < nks; ++ks) {
          double fn[NSL][4];
          load(min(ks + 1, nks - 1), fn);
#pragma unroll
          for (int s = 0; s < NSL; ++s)
            acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[s][0] * f[s][1], f[s][2] * f[s][3], acc[s], 0, 0, 0);
          if (bot0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int pt = 4 * ks + split + j;
              if ((j & (nsplit - 1)) == 0 && pt < nc) bottom_point0(pt);
            }
          }
#pragma unroll
          for (int s = 0; s < NSL; ++s)
#pragma unroll
            for (int j = 0; j < 4; ++j) f[s][j] = fn[s][j];
        }
      };
      switch (nslot0) {
        case 1: top_tiles(std::integral_constant<int, 1>{}); break;
        case 2: top_tiles(std::integral_constant<int, 2>{}); break;
        case 3: top_tiles(std::integral_constant<int, 3>{}); break;
        case 4: top_tiles(std::integral_constant<int, 4>{}); break;
        case 5: top_tiles(std::integral_constant<int, 5>{}); break;
        default: top_tiles(std::integral_constant<int, kMomTileSlots>{}); break;
      }
      // bottom moments (monomials of degree <= p), VALU tasks: slot 0 (inside the
      // top-tile steps above) keeps its sums over all chunks, later slots (only
      // with nsplit = 1) add theirs now
#pragma unroll
      for (int sl = 1; sl < kTaskSlots1; ++sl) {
        if (ttask + sl * span >= ntask1) break;
        double bu[4], bv[4][NS + 1];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          bu[c] = 0.0;
#pragma unroll
          for (int q = 0; q <= NS; ++q) bv[c][q] = 0.0;
        }
        bottom_sums(sl, nc, bu, bv);
        bottom_flush(sl, bu, bv);
      }
      __syncthreads();
    }
    // after the element's last chunk: fold its tiles (each moment index belongs
    // to one tile entry, so no two lanes or waves write the same word)
    if (cc % cpe == cpe - 1) {
      double g[NS];
#pragma unroll
      for (int d = 0; d < NS; ++d) g[d] = R[El<NS>::GNEW + d];
#pragma unroll
      for (int s = 0; s < kMomTileSlots; ++s) {
        const int t = wave + 4 * s;
        if (t < ntile) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int b = mt_map[t * 256 + ((lane >> 4) + 4 * r) * 16 + (lane & 15)];
            if (b >= 0) {
              const double c = acc[s][r];
              NU[b] += c;
#pragma unroll
              for (int d = 0; d < NS; ++d) NU[(1 + d) * M2 + b] += g[d] * c;
            }
          }
        }
        acc[s] = d4{0.0, 0.0, 0.0, 0.0};
      }
    }
  }
  __syncthreads();
  // slot 0's sums of the groups, group by group
  for (int s = 0; s < nsplit; ++s) {
    if (split == s && ttask < ntask1) bottom_flush(0, bu0, bv0);
    __syncthreads();
  }
  // the recovery row's weight and U sums: each set-up thread's, then the block's
  block_sum2(sw_acc, su_acc, PW);
  if (tid == 0) {
    *A00r += sw_acc;
    *r0r += su_acc;
  }
}

// Fields of the solution at one point from the monomial runs of the degree-p
// table: val[c] += sum_k cm[c*M + k] m_k(var) for c <= NS over the monomials of
// degree <= p-1 (v, sigma), and with WITH_U val[NS+1] over all monomials (U).
// var = (th, xh_1..xh_n); the run loop and the coefficient addresses are the same
// for every thread.
template <int NS, bool WITH_U>
__device__ inline void eval_runs(const Tab& T, const int* runs, const double* var, const double* cm, double* val) {
  const int M = T.M, M1 = T.M1;
  const double z = var[NS];
  for (int t = 0; t < T.ntask1; ++t) {
    const unsigned w0 = (unsigned)runs[t * kTaskInts];
    const unsigned w1 = (unsigned)runs[t * kTaskInts + 1];
    const unsigned w2 = (unsigned)runs[t * kTaskInts + 2];
    double mv = 1.0;
#pragma unroll
    for (int v = 0; v < NS; ++v) {
      const int ev = (int)((w0 >> (5 * v)) & 31u);
      for (int i = 0; i < ev; ++i) mv *= var[v];
    }
    const int d0 = (int)((w0 >> 15) & 31u);
    for (int i = 0; i < d0; ++i) mv *= z;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const unsigned ww = c < 2 ? w1 : w2;
      const int k = (int)((c & 1) ? (ww >> 16) : (ww & 0xFFFFu));
      if (k == 0xFFFF) break;
      if (k < M1) {
#pragma unroll
        for (int comp = 0; comp <= NS; ++comp) val[comp] += cm[comp * M + k] * mv;
      }
      if (WITH_U) val[NS + 1] += cm[(NS + 1) * M + k] * mv;
      mv *= z;
    }
  }
}

// Fields of a solution at 16 points per wave on the FP64 matrix cores (3+1D).
// A monomial of degree <= p is L_a(th, xh1) R_b(xh2, xh3) (entries a, b of the
// two-variable list EX, by degree), so field c at point pt is
//   val_c(pt) = sum_a L_a(pt) Y_c[pt][a],   Y_c[pt][a] = sum_b R_b(pt) CM_c[a][b],
// with CM_c the dense coefficients (rows a < nA16, row stride ldb).  Y is a
// 16x16x4 MFMA chain per tile of 16 entries a (A: R_b at point l%16, entry b =
// 4 ks + l/16; B: CM_c[a = 16 I + l%16][b]); tile I needs nks[I] steps (the
// entries b of degree <= p minus the tile's smallest degree), and nkv[I] for
// the first NV fields (v and sigma: degree <= p - 1; the steps past nkv[I]
// would only add exact zeros).  Each lane then
// weights its four results (points l/16 + 4r, entry 16 I + l%16) by L_a and
// the 16 lanes of a row are summed (DPP): every lane of row l/16 ends with val[c][r]
// of point l/16 + 4r.  PWW: powers of the wave's 16 points, PWW[(pt*4 + v)*P1
// + e] = var_v^e (v = 0: th).
template <int NC, int NV>
__device__ inline void eval16_mfma(const double* CMd, int nA16, int ldb, int nl, int nat, const int* nks,
                                   const int* nkv, const int* EX, const double* PWW, int P1,
                                   double (&val)[NC][4]) {
  constexpr int KMAX = kEvalMaxSteps;
  const int lane = threadIdx.x & 63;
  const int pi = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) val[c][r] = 0.0;
  // the A operands R_b(point pi), b = 4 ks + kq, once for every field and tile
  // (tile 0 needs the most steps)
  const int nk0 = NV < NC ? nks[0] : nkv[0];
  double rv[KMAX];
  {
    const double* pw = PWW + pi * 4 * P1;
#pragma unroll
    for (int ks = 0; ks < KMAX; ++ks) {
      const int b = ks * 4 + kq;
      rv[ks] = 0.0;
      if (ks < nk0 && b < nl) {
        const int eb = EX[b];
        rv[ks] = pw[2 * P1 + (eb & 255)] * pw[3 * P1 + (eb >> 8)];
      }
    }
  }
  for (int I = 0; I < nat; ++I) {
    const int a = I * 16 + pi;
    const int ea = a < nl ? EX[a] : 0;
    double La[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double* pw = PWW + (kq + 4 * r) * 4 * P1;
      La[r] = a < nl ? pw[ea & 255] * pw[P1 + (ea >> 8)] : 0.0;
    }
    const int nkvI = nkv[I];
    const int nk = NV < NC ? nks[I] : nkvI;
    d4 acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
    // the fields' chains interleaved (independent accumulators)
#pragma unroll
    for (int ks = 0; ks < KMAX; ++ks) {
      if (ks < nk) {
        const int b = ks * 4 + kq;
        const bool sv = ks < nkvI;  // the first NV fields (degree <= p - 1) need fewer steps
        double bv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c)
          bv[c] = (b < nl && (c >= NV || sv)) ? CMd[((long long)c * nA16 + a) * ldb + b] : 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c)
          if (c >= NV || sv) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(rv[ks], bv[c], acc[c], 0, 0, 0);
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) val[c][r] += acc[c][r] * La[r];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) val[c][r] = row16_sum(val[c][r]);
}

// eval16_mfma at two times per point: every point has 5 power rows (P1 each:
// th at the bottom, xh_1..xh_3, th at the top), the products Y_c[pt][a] are
// formed once, and valb[c] (c < NB, the bottom time) and valt[c] (all NC
// fields, the top time) are its sums against L_a at either time.  KMAX >= the
// step count of tile 0.
template <int NC, int NV, int NB, int KMAX>
__device__ inline void eval16_mfma2(const double* CMd, int nA16, int ldb, int nl, int nat, const int* nks,
                                    const int* nkv, const int* EX, const double* PWW, int P1,
                                    double (&valb)[NB][4], double (&valt)[NC][4]) {
  const int lane = threadIdx.x & 63;
  const int pi = lane & 15, kq = lane >> 4;
  const int ps = 5 * P1;
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) valt[c][r] = 0.0;
#pragma unroll
  for (int c = 0; c < NB; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) valb[c][r] = 0.0;
  const int nk0 = nks[0];
  double rv[KMAX];
  {
    const double* pw = PWW + pi * ps;
#pragma unroll
    for (int ks = 0; ks < KMAX; ++ks) {
      const int b = ks * 4 + kq;
      rv[ks] = 0.0;
      if (ks < nk0 && b < nl) {
        const int eb = EX[b];
        rv[ks] = pw[2 * P1 + (eb & 255)] * pw[3 * P1 + (eb >> 8)];
      }
    }
  }
  for (int I = 0; I < nat; ++I) {
    const int a = I * 16 + pi;
    const int ea = a < nl ? EX[a] : 0;
    double Lb[4], Lt[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double* pw = PWW + (kq + 4 * r) * ps;
      Lb[r] = a < nl ? pw[ea & 255] * pw[P1 + (ea >> 8)] : 0.0;
      Lt[r] = a < nl ? pw[4 * P1 + (ea & 255)] * pw[P1 + (ea >> 8)] : 0.0;
    }
    const int nkvI = nkv[I];
    const int nk = nks[I];
    d4 acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KMAX; ++ks) {
      if (ks < nk) {
        const int b = ks * 4 + kq;
        const bool sv = ks < nkvI;
        double bv[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c)
          bv[c] = (b < nl && (c >= NV || sv)) ? CMd[((long long)c * nA16 + a) * ldb + b] : 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c)
          if (c >= NV || sv) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(rv[ks], bv[c], acc[c], 0, 0, 0);
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        valt[c][r] += acc[c][r] * Lt[r];
        if (c < NB) valb[c < NB ? c : 0][r] += acc[c][r] * Lb[r];
      }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) valt[c][r] = row16_sum(valt[c][r]);
#pragma unroll
  for (int c = 0; c < NB; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) valb[c][r] = row16_sum(valb[c][r]);
}

// Dense coefficients CM_c[a][b] of the fields of group r's solution xs (3+1D):
// the transposed table contracted with the coefficients, scattered by ev_ab;
// the U row scaled by h (U_j = h Uhat_j).  Whole workgroup; ends with a barrier.
template <int NS>
__device__ inline void build_cm_dense(const Tab& T, const TableDesc& Dp, const double* xr, double hr, double* CMd,
                                      int nA16, int ldb) {
  const int tid = threadIdx.x;
  for (int i = tid; i < (NS + 2) * nA16 * ldb; i += blockDim.x) CMd[i] = 0.0;
  __syncthreads();
  for (int row = tid; row < (NS + 2) * T.M; row += blockDim.x) {
    double acc = 0.0;
    for (int e = T.tr_ptr[row]; e < T.tr_ptr[row + 1]; ++e) acc += T.tr_coef[e] * xr[T.tr_j[e]];
    const int comp = row / T.M, k = row % T.M;
    const int ab = Dp.ev_ab[k];
    CMd[((long long)comp * nA16 + (ab & 0xFFFF)) * ldb + (ab >> 16)] = comp == NS + 1 ? acc * hr : acc;
  }
  __syncthreads();
}

template <int NS, int TPW, bool MIXED, bool MOM>
__device__ __attribute__((always_inline)) void solve_tent(const KParams& P, const LdsPlan& L, const int tent, double* lds) {
  __shared__ int s_m, s_piv, s_err, s_goff[kMaxGroups + 1], s_conv;
  __shared__ double s_red[2 * kBlock / 64];
  __shared__ int s_gel[kMaxPatch];
  __shared__ int s_fl[kMaxFaces], s_foff[kMaxGroups + 1];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int V = P.tent_V[tent];
  const double tb = P.tent_tb[tent], tt = P.tent_tt[tent];
  const double tmid = 0.5 * (tb + tt);
  const double dt = tt - tb;
  const int p_in = P.p_per_tent ? (int)P.p_per_tent[tent] : (P.p_fixed > 0 ? P.p_fixed : P.pmax);
  const int pb = P.v2e_ptr[V];
  const int npatch = P.v2e_ptr[V + 1] - pb;
  const int Q = P.Q;
  const int ELS = L.ELS;
  if (p_in < 1 || p_in > P.pmax || npatch > L.maxpatch) {
    if (tid == 0) atomicOr(P.status, (p_in < 1 || p_in > P.pmax) ? kStatSize : kStatPatch);
    return;
  }
  // ---- LDS carve-up --------------------------------------------------------------
  double* xs = lds + L.off_x;
  double* EL = lds + L.off_el;
  double* MS = lds + L.off_misc;
  double* gc = MS;
  double* gh = gc + kMaxGroups;
  double* A00 = gh + kMaxGroups;
  double* r0 = A00 + kMaxGroups;
  double* a0 = r0 + kMaxGroups;
  double* fsc = a0 + kMaxGroups;  // 24: face measure, normal, simplex vertices
  double* A0 = fsc + 24;          // (groups of the mesh's largest patch) x NWP
  // system: LDS or this workgroup's slot of the global scratch
  const long long lda = L.lda;
  double* A = L.A_in_lds ? lds + L.off_A : P.work + (long long)blockIdx.x * P.work_stride;

  // A tent solved at a degree below p_max whose realised indicator exceeds the
  // tolerance is solved again one degree higher (at most up to p_max, where it
  // is accepted); nothing is written before the accepted attempt.
  for (int dtry = 0;; ++dtry) {
  const int p = min(p_in + dtry, P.pmax);
  // chunk size and operand stride of degree p (lower degrees take larger chunks)
  const TableDesc& Dp = P.tabd[p];
  const int PCH = Dp.pch;
  const int LD2 = 2 * PCH;  // row stride of the monomial table (top points, then bottom points)
  const int NWP = Dp.nwp;
  double* PV = lds + L.off_pt;    // 2*PCH x (NS+1): top then bottom coordinates
  double* PW = PV + 2 * PCH * (NS + 1);  // PCH weights
  double* PD = PW + PCH;                 // PCH x (NS+2): weighted bottom data, w*U_b
  double* PG = PD + PCH * (NS + 2);      // PCH x NS: grad phi_new at the point
  double* PS = PG + PCH * NS;            // PCH: c^-2 - |g_new|^2
  double* POW = lds + L.off_pow;         // 2*PCH x (NS+1) x (p+1)
  double* W1 = lds + L.off_W1;           // PSI: PCH*(NS+1) rows, RB: PCH rows, UB: PCH rows (row stride NWP)
  // M x 2*PCH monomials (top points, then bottom points) of the quadrature Gram
  double* MT = MOM ? nullptr : lds + L.off_mono;
  const int PCI = Dp.pci;  // points per chunk of the interface faces
  double* PSI = W1;
  double* RB = W1 + PCH * (NS + 1) * NWP;
  double* UB = RB + PCH * NWP;
  // ---- table of degree p (staged in LDS when it fits) ----------------------------
  Tab T;
  {
    const TableDesc& D = Dp;
    T.NW = D.NW;
    T.M = D.M;
    T.M1 = D.M1;
    T.M2 = D.M2;
    T.fo_ptr = D.fo_ptr;
    T.fo_idx = D.fo_idx;
    T.fo_coef = D.fo_coef;
    T.u_ptr = D.u_ptr;
    T.u_idx = D.u_idx;
    T.u_coef = D.u_coef;
    T.expo2 = D.expo2;
    T.K2 = D.K2;
    T.task2 = D.task2;
    T.task1 = D.task1;
    T.ntask2 = D.ntask2;
    T.ntask1 = D.ntask1;
    if (L.tab_in_lds) {
      const int nue = D.ue_n, ntr = D.tr_n, nrow = (NS + 2) * D.M;
      int* ti = reinterpret_cast<int*>(lds + L.off_tab);
      double* td = lds + L.off_tab + L.tab_int_dbl;
      int* t_up = ti;
      int* t_ui = t_up + (D.NW + 1);
      int* t_tp = t_ui + nue * (NS + 2);
      int* t_tj = t_tp + nrow + 1;
      int* t_ex = t_tj + ntr;
      double* t_uc = td;
      double* t_tc = td + nue * (NS + 2);
      for (int i = tid; i <= D.NW; i += blockDim.x) t_up[i] = D.ue_ptr[i];
      for (int i = tid; i < nue * (NS + 2); i += blockDim.x) {
        t_ui[i] = D.ue_idx[i];
        t_uc[i] = D.ue_coef[i];
      }
      for (int i = tid; i <= nrow; i += blockDim.x) t_tp[i] = D.tr_ptr[i];
      for (int i = tid; i < ntr; i += blockDim.x) {
        t_tj[i] = D.tr_j[i];
        t_tc[i] = D.tr_coef[i];
      }
      for (int i = tid; i < D.M * (NS + 1); i += blockDim.x) t_ex[i] = D.expo[i];
      T.ue_ptr = t_up;
      T.ue_idx = t_ui;
      T.ue_coef = t_uc;
      T.tr_ptr = t_tp;
      T.tr_j = t_tj;
      T.tr_coef = t_tc;
      T.expo = t_ex;
    } else {
      T.ue_ptr = D.ue_ptr;
      T.ue_idx = D.ue_idx;
      T.ue_coef = D.ue_coef;
      T.tr_ptr = D.tr_ptr;
      T.tr_j = D.tr_j;
      T.tr_coef = D.tr_coef;
      T.expo = D.expo;
    }
  }
  const int NW = T.NW;
  const double* XV = P.coords + (size_t)V * NS;

  // ---- 1. patch records, speed groups, diameters ---------------------------------
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
    // element lists per group, in patch order
    int c = 0;
    for (int r = 0; r < m; ++r) {
      s_goff[r] = c;
      for (int i = 0; i < npatch; ++i)
        if ((int)EL[i * ELS + El<NS>::GRP] == r) s_gel[c++] = i;
    }
    s_goff[m] = c;
    s_m = m;
  }
  __syncthreads();
  const int m = s_m;
  // recover_U = 2 (Sec. 5, every test function): the constants of the groups
  // are unknowns S0 .. S0+m-1 after the functions; the right-hand side is column S
  const bool R2 = P.recover_U == 2;
  const int S0 = m * NW;
  const int S = S0 + (R2 ? m : 0);
  if (s_err || S > L.S || (MOM && R2)) {
    if (tid == 0) atomicOr(P.status, s_err ? s_err : kStatSize);
    return;
  }
  // group diameters h_r (eq. 3.3 with the group's speed), eight groups per pass
  for (int r0g = 0; r0g < m; r0g += 8) {
    const int nvert = npatch * (NS + 1) + 1;
    const long long npair = (long long)nvert * (nvert - 1) / 2;
    double hloc[8];
    for (int r = 0; r < 8; ++r) hloc[r] = 0.0;
    for (long long pi = tid; pi < npair; pi += blockDim.x) {
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
#pragma unroll
      for (int r = 0; r < 8; ++r)
        if (r0g + r < m) hloc[r] = fmax(hloc[r], sqrt(dx2 + gc[r0g + r] * gc[r0g + r] * dtt * dtt));
    }
#pragma unroll
    for (int r = 0; r < 8; ++r)
      if (r0g + r < m) atomic_max_nonneg(&gh[r0g + r], hloc[r]);
  }
  // mixed precision: FP32 Gram first; faces kept apart (AF) for the FP64 residual
  double* AF = nullptr;
  double* bvec = nullptr;  // right-hand side before elimination
  double* rvec = nullptr;  // residual / correction
  if constexpr (MIXED) {
    AF = L.A_in_lds ? lds + L.off_AF : A + (long long)L.S * lda;
    bvec = lds + L.off_vec;
    rvec = bvec + L.S;
  }
  bool use32 = MIXED;
  int ir_steps = 0;
  for (int attempt = 0;; ++attempt) {
  for (long long i = tid; i < (long long)S * lda; i += blockDim.x) {
    A[i] = 0.0;
    if constexpr (MIXED) AF[i] = 0.0;
  }
  for (int i = tid; i < m * NWP; i += blockDim.x) A0[i] = 0.0;
  if (tid < kMaxGroups) {
    A00[tid] = 0.0;
    r0[tid] = 0.0;
  }
  __syncthreads();

  if constexpr (MOM) {
    // ---- 2'. top Gram, bottom right-hand side and recovery rows from moments ------
    // The fields are sparse combinations of the monomials m_k, k < M1, so over the
    // top points  sum_q w [v_i v_j/c^2 + s_i.s_j - (v_i s_j + v_j s_i).g]  is a
    // combination of the moments nu[b] = sum_q w m_b and nu_d[b] = sum_q w g_d m_b
    // of the monomials b of degree <= 2p-2 (products m_k m_l = m_K2(k,l)); the
    // right-hand side and the recovery row need the moments of m_k over the bottom
    // points weighted by the incoming data.
    const Tab& D = T;
    const int M2 = T.M2, M1 = T.M1, Mm = T.M;
    const int E2 = 2 * p - 1;  // top powers 0 .. 2p-2
    double* NU = W1;                    // (NS+1) x M2: nu, nu_1..nu_n
    double* BV = NU + (NS + 1) * M2;    // (NS+1) x M1: bottom moments times the data
    double* BU = BV + (NS + 1) * M1;    // M: bottom moments sum w m_k
    double* POWT = POW;
    double* POWB = POW + PCH * (NS + 1) * E2;
    for (int r = 0; r < m; ++r) {
      const double cr = gc[r], hr = gh[r];
      const double ic2 = 1.0 / (cr * cr);
      const int npts = (s_goff[r + 1] - s_goff[r]) * Q;
      bool done_mt = false;
      if constexpr (NS == 3) {
        if (Dp.mt_ntile > 0) {
          // a lower degree may take a larger chunk in the free tail of W1
          int mpch = PCH;
          double *mPV = PV, *mPW = PW, *mPD = PD, *mPOWT = POWT, *mPOWB = POWB;
          if (Dp.moff >= 0) {
            mpch = Dp.mpch;
            mPV = W1 + Dp.moff;
            mPW = mPV + 2 * mpch * (NS + 1);
            mPD = mPW + mpch;
            mPOWT = mPD + mpch * (NS + 2);
            mPOWB = mPOWT + mpch * (NS + 1) * E2;
          }
          moment_points_mt<NS>(P.lam_ref, P.w_ref, P.state, Q, EL, ELS, s_gel + s_goff[r], s_goff[r + 1] - s_goff[r],
                               XV, cr, hr, tmid, dt, p, mpch, M1, M2, Mm, T.task1, T.ntask1, Dp.mt_ntile, Dp.mt_ex,
                               Dp.mt_map, NU, BV, BU, mPV, mPW, mPD, mPOWT, mPOWB, A00 + r, r0 + r);
          done_mt = true;
        }
      }
      if (!done_mt)
        moment_points<NS>(P.lam_ref, P.w_ref, P.state, Q, EL, ELS, s_gel + s_goff[r], npts, XV, cr, hr, tmid, dt, p,
                          PCH, M1, M2, Mm, T.task1, T.ntask1, T.task2, T.ntask2, NU, BV, BU, PV, PW, PD, PG, POWT,
                          POWB, A00 + r, r0 + r);
      // right-hand side and recovery row of group r
      for (int i = tid; i < NW; i += blockDim.x) {
        double b = 0.0;
        for (int a = 0; a <= NS; ++a) {
          const int row = i * (NS + 1) + a;
          const double sc = a == 0 ? cr : 1.0;
          for (int e = D.fo_ptr[row]; e < D.fo_ptr[row + 1]; ++e) b += D.fo_coef[e] * sc * BV[a * M1 + D.fo_idx[e]];
        }
        A[(long long)(r * NW + i) * lda + S] += b;
        double u = 0.0;
        for (int e = D.u_ptr[i]; e < D.u_ptr[i + 1]; ++e) u += D.u_coef[e] * BU[D.u_idx[e]];
        A0[r * NWP + i] += hr * u;
      }
      __syncthreads();
      // Gram block (r, r) from the moments (Z reuses the bottom moments' space)
      moment_gram_block<NS>(T.fo_ptr, T.fo_idx, T.fo_coef, T.K2, M1, M2, NW, NU, BV,
                            (long long)(L.off_fg - L.off_W1) - (long long)(NS + 1) * M2, cr, 0.0, false, A, lda,
                            r * NW);
    }
  } else {
  // ---- 2. top Gram (matrix cores), bottom right-hand side, U recovery rows --------
  const int ntile_dim = (NW + 15) / 16;
  const int ntiles = ntile_dim * (ntile_dim + 1) / 2;
  const int padc = ntile_dim * 16 - NW;
  // lower-triangular Gram tiles (I >= J); a pass over the points accumulates
  // kBlock/64 * TPW of them in registers, more tiles take more passes
  const int tiles_per_pass = (kBlock / 64) * TPW;
  const int npass = (ntiles + tiles_per_pass - 1) / tiles_per_pass;
  for (int rp = 0; rp < m * npass; ++rp) {
    const int r = rp / npass, pass = rp % npass;
    const double cr = gc[r], hr = gh[r];
    const int npts = (s_goff[r + 1] - s_goff[r]) * Q;
    int tI[TPW], tJ[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tile = pass * tiles_per_pass + wave * TPW + t;
      int I = 0;
      while ((I + 1) * (I + 2) / 2 <= tile) ++I;
      tI[t] = tile < ntiles ? I : -1;
      tJ[t] = tile - I * (I + 1) / 2;
    }
    d4 acc[TPW];
    f4 acc32[MIXED ? TPW : 1];
#pragma unroll
    for (int t = 0; t < TPW; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < (MIXED ? TPW : 1); ++t) acc32[t] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    float* PSI32 = reinterpret_cast<float*>(PSI);
    double rhs_acc = 0.0, a0_acc = 0.0;    // column j = tid
    double rhs_acc2 = 0.0, a0_acc2 = 0.0;  // column j = tid + blockDim.x
    double sw_acc = 0.0, su_acc = 0.0;     // recovery row: this thread's set-up points
    for (int f0 = 0; f0 < npts; f0 += PCH) {
      const int nc = min(PCH, npts - f0);
      // point set-up
      for (int pt = tid; pt < PCH; pt += blockDim.x) {
        double xt[NS], g[NS], dd[NS + 2];
        double phi = tmid, pho = tmid, w = 0.0, sD = 0.0;
        for (int k = 0; k < NS + 2; ++k) dd[k] = 0.0;
        for (int d = 0; d < NS; ++d) {
          xt[d] = XV[d];
          g[d] = 0.0;
        }
        if (pt < nc) {
          const int f = f0 + pt;
          const int li = s_gel[s_goff[r] + f / Q];
          const int q = f % Q;
          const double* R = EL + li * ELS;
          const int lV = (int)R[El<NS>::LV];
          const int e = (int)R[El<NS>::E];
          const double* lam = P.lam_ref + (size_t)q * (NS + 1);
          pho = 0.0;
          for (int d = 0; d < NS; ++d) xt[d] = 0.0;
          for (int k = 0; k <= NS; ++k) {
            pho += lam[k] * R[El<NS>::TAU + k];
            for (int d = 0; d < NS; ++d) xt[d] += lam[k] * R[El<NS>::X + k * NS + d];
          }
          phi = pho + lam[lV] * dt;
          w = P.w_ref[q] * R[El<NS>::DET];
          const double ic2 = 1.0 / (cr * cr);
          double gn2 = 0.0;
          for (int d = 0; d < NS; ++d) {
            g[d] = R[El<NS>::GNEW + d];
            gn2 += g[d] * g[d];
          }
          sD = ic2 - gn2;
          const double* st = P.state + (size_t)e * (NS + 2) * Q;
          const double vb = st[q];
          double sg = 0.0;
          for (int d = 0; d < NS; ++d) sg += st[(1 + d) * Q + q] * R[El<NS>::GOLD + d];
          dd[0] = w * (ic2 * vb - sg);
          for (int d = 0; d < NS; ++d) dd[1 + d] = w * (st[(1 + d) * Q + q] - vb * R[El<NS>::GOLD + d]);
          dd[NS + 1] = w * st[(NS + 1) * Q + q];
        }
        PV[pt * (NS + 1)] = cr * (phi - tmid) / hr;
        PV[(PCH + pt) * (NS + 1)] = cr * (pho - tmid) / hr;
        for (int d = 0; d < NS; ++d) {
          const double xh = (xt[d] - XV[d]) / hr;
          PV[pt * (NS + 1) + 1 + d] = xh;
          PV[(PCH + pt) * (NS + 1) + 1 + d] = xh;
          PG[pt * NS + d] = g[d];
        }
        PW[pt] = w;
        PS[pt] = sD;
        for (int k = 0; k < NS + 2; ++k) PD[pt * (NS + 2) + k] = dd[k];
        sw_acc += w;
        su_acc += dd[NS + 1];
      }
      __syncthreads();
      // powers and monomials of the top and bottom points
      monomials<NS>(T, T.M, p, PV, POW, MT, LD2, 2 * PCH);
      __syncthreads();
      // fields: flat over (point, function)
      for (int i = tid; i < PCH * NW; i += blockDim.x) {
        const int pt = i % PCH, j = i / PCH;
        const double w = PW[pt];
        const double sw = sqrt(w), swD = sqrt(w * PS[pt]);
        double f[NS + 1], fb[NS + 1], ub = 0.0;
        eval_j<NS, false>(T, j, MT, LD2, pt, f, &ub);
        if (pass == 0 || R2) eval_j<NS, true>(T, j, MT, LD2, PCH + pt, fb, &ub);
        const double v = cr * f[0];
        if (MIXED && use32) {
          float* row = PSI32 + (size_t)pt * (NS + 1) * NWP + j;
          row[0] = (float)(swD * v);
          for (int d = 0; d < NS; ++d) row[(1 + d) * NWP] = (float)(sw * (f[1 + d] - PG[pt * NS + d] * v));
        } else {
          double* row = PSI + (size_t)pt * (NS + 1) * NWP + j;
          row[0] = swD * v;
          for (int d = 0; d < NS; ++d) row[(1 + d) * NWP] = sw * (f[1 + d] - PG[pt * NS + d] * v);
        }
        if (pass == 0) {
          double accb = cr * fb[0] * PD[pt * (NS + 2)];
          for (int d = 0; d < NS; ++d) accb += fb[1 + d] * PD[pt * (NS + 2) + 1 + d];
          // R2: int_bot U_bot U_i joins the right-hand side of function i
          if (R2) accb += PD[pt * (NS + 2) + NS + 1] * hr * ub;
          RB[pt * NWP + j] = accb;
        }
        // recovery row sum_q w U_j, or (R2) sqrt(w) U_j: the rows of the bottom
        // mass Gram sum_q w U_i U_j, formed on the matrix cores with the top Gram
        if (pass == 0 || R2) UB[pt * NWP + j] = (R2 ? sqrt(w) : w) * hr * ub;
      }
      // zero the padding columns of PSI so the 16-wide tiles see zeros
      for (int i = tid; i < PCH * (NS + 1) * padc; i += blockDim.x) {
        const int row = i / padc, col = NW + i % padc;
        if (MIXED && use32)
          PSI32[row * NWP + col] = 0.0f;
        else
          PSI[row * NWP + col] = 0.0;
      }
      if (R2)
        for (int i = tid; i < PCH * padc; i += blockDim.x) UB[(i / padc) * NWP + NW + i % padc] = 0.0;
      __syncthreads();
      // Gram on the matrix cores: lane l of a k-step reads row 4 ks + l/16, column 16 I + l%16
      {
        const int nk = (nc * (NS + 1) + 3) / 4;
        if (MIXED && use32) {
          for (int ks = 0; ks < nk; ++ks) {
            const float* rowp = PSI32 + (size_t)(ks * 4 + (lane >> 4)) * NWP + (lane & 15);
#pragma unroll
            for (int t = 0; t < (MIXED ? TPW : 1); ++t)
              if (tI[t] >= 0)
                acc32[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(rowp[tI[t] * 16], rowp[tJ[t] * 16], acc32[t], 0, 0, 0);
          }
        } else {
          for (int ks = 0; ks < nk; ++ks) {
            const double* rowp = PSI + (size_t)(ks * 4 + (lane >> 4)) * NWP + (lane & 15);
#pragma unroll
            for (int t = 0; t < TPW; ++t)
              if (tI[t] >= 0)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(rowp[tI[t] * 16], rowp[tJ[t] * 16], acc[t], 0, 0, 0);
          }
          // R2: bottom mass sum_q w U_i U_j (rows sqrt(w) U of the chunk's points;
          // rows past nc hold zero weights, PCH is a multiple of 4)
          if (R2)
            for (int ks = 0; ks < (nc + 3) / 4; ++ks) {
              const double* rowp = UB + (size_t)(ks * 4 + (lane >> 4)) * NWP + (lane & 15);
#pragma unroll
              for (int t = 0; t < TPW; ++t)
                if (tI[t] >= 0)
                  acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(rowp[tI[t] * 16], rowp[tJ[t] * 16], acc[t], 0, 0, 0);
            }
        }
      }
      // right-hand side and recovery row: column sums over the chunk's points
      for (int j = tid; j < (pass == 0 ? NW : 0); j += blockDim.x) {
        double s1 = 0.0, s2 = 0.0;
        for (int pt = 0; pt < nc; ++pt) {
          s1 += RB[pt * NWP + j];
          s2 += R2 ? sqrt(PW[pt]) * UB[pt * NWP + j] : UB[pt * NWP + j];
        }
        if (j == tid) {
          rhs_acc += s1;
          a0_acc += s2;
        } else {
          rhs_acc2 += s1;
          a0_acc2 += s2;
        }
      }
      __syncthreads();
    }
    // Gram tiles of block (r, r): element e of lane l is row l/16 + 4e, column l%16
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      if (tI[t] >= 0) {
        const int I = tI[t], J = tJ[t];
        const int j = J * 16 + (lane & 15);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          // FP64 output: row l/16 + 4e; FP32 output: row 4(l/16) + e; column l%16
          const bool f32 = MIXED && use32;
          const int i = I * 16 + (f32 ? 4 * (lane >> 4) + e : (lane >> 4) + 4 * e);
          double val;
          if constexpr (MIXED)
            val = f32 ? (double)acc32[t][e] : acc[t][e];
          else
            val = acc[t][e];
          if (i < NW && j < NW) {
            A[(long long)(r * NW + i) * lda + r * NW + j] += val;
            if (I != J) A[(long long)(r * NW + j) * lda + r * NW + i] += val;
          }
        }
      }
    }
    if (pass == 0) {
      // the recovery row's weight and U sums: each set-up thread's, then the block's
      block_sum2(sw_acc, su_acc, s_red);
      if (tid == 0) {
        A00[r] += sw_acc;
        r0[r] += su_acc;
      }
    }
    if (pass == 0 && tid < NW) {
      A[(long long)(r * NW + tid) * lda + S] += rhs_acc;
      A0[r * NWP + tid] += a0_acc;
    }
    if (pass == 0 && tid + (int)blockDim.x < NW) {
      A[(long long)(r * NW + tid + blockDim.x) * lda + S] += rhs_acc2;
      A0[r * NWP + tid + blockDim.x] += a0_acc2;
    }
    __syncthreads();
  }

  }  // quadrature Gram
  if (R2) {
    // the constant's row (test function 1) and column (trial constant) of each
    // group: sum_q w U_j, sum_q w, and the right-hand side sum_q w U_bot
    for (int i = tid; i < m * NW; i += blockDim.x) {
      const int r = i / NW, j = i % NW;
      const double v = A0[r * NWP + j];
      A[(long long)(S0 + r) * lda + r * NW + j] = v;
      A[(long long)(r * NW + j) * lda + S0 + r] = v;
    }
    if (tid < m) {
      A[(long long)(S0 + tid) * lda + S0 + tid] = A00[tid];
      A[(long long)(S0 + tid) * lda + S] = r0[tid];
    }
    __syncthreads();
  }

  // ---- 3. time-like faces above facets containing V ---------------------------------
  const int nbf = P.vb_ptr[V + 1] - P.vb_ptr[V];
  const int nif = P.vi_ptr[V + 1] - P.vi_ptr[V];
  double* F1 = W1;  // 4 x PCH rows of NWP: face values
  double* AT = MIXED ? AF : A;  // face terms (kept apart in the mixed path)
  if (nbf > L.maxfaces) {
    if (tid == 0) atomicOr(P.status, kStatSize);
    return;
  }
  // 3a. Dirichlet faces: geometry of every face, then all face points of a
  //     speed group in one chunked pass
  constexpr int FGS = 2 + NS + (NS + 1) * (NS + 1);  // measure, group, normal, simplex vertices
  double* FG = lds + L.off_fg;
  for (int f = tid; f < nbf; f += blockDim.x) {
    const int e1 = P.vb[2 * (P.vb_ptr[V] + f)];
    const int k1 = P.vb[2 * (P.vb_ptr[V] + f) + 1];
    double* G0 = FG + f * FGS;
    const int* vs = P.elems + (size_t)e1 * (NS + 1);
    double Pv[NS + 1][NS + 1];
#pragma unroll
    for (int d = 0; d < NS; ++d) {
      Pv[0][d] = XV[d];
      Pv[1][d] = XV[d];
    }
    Pv[0][NS] = tb;
    Pv[1][NS] = tt;
    int c = 2;
#pragma unroll
    for (int k = 0; k <= NS; ++k) {
      const int w = vs[k];
      if (k == k1 || w == V) continue;
#pragma unroll
      for (int i = 2; i <= NS; ++i)
        if (i == c) {
          for (int d = 0; d < NS; ++d) Pv[i][d] = P.coords[(size_t)w * NS + d];
          Pv[i][NS] = P.tau[w];
        }
      ++c;
    }
    double E[NS][NS + 1], Gm[NS][NS];
#pragma unroll
    for (int i = 0; i < NS; ++i)
#pragma unroll
      for (int d = 0; d <= NS; ++d) E[i][d] = Pv[i + 1][d] - Pv[0][d];
#pragma unroll
    for (int i = 0; i < NS; ++i)
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        double sacc = 0.0;
#pragma unroll
        for (int d = 0; d <= NS; ++d) sacc += E[i][d] * E[j][d];
        Gm[i][j] = sacc;
      }
    double detG;
    if (NS == 1)
      detG = Gm[0][0];
    else if (NS == 2)
      detG = Gm[0][0] * Gm[1][1] - Gm[0][1] * Gm[1][0];
    else
      detG = Gm[0][0] * (Gm[1][1] * Gm[2][2] - Gm[1][2] * Gm[2][1]) -
             Gm[0][1] * (Gm[1][0] * Gm[2][2] - Gm[1][2] * Gm[2][0]) +
             Gm[0][2] * (Gm[1][0] * Gm[2][1] - Gm[1][1] * Gm[2][0]);
    G0[0] = sqrt(fmax(detG, 0.0));
    int g1 = 0;
    for (int i = 0; i < npatch; ++i)
      if ((int)EL[i * ELS + El<NS>::E] == e1) g1 = (int)EL[i * ELS + El<NS>::GRP];
    G0[1] = (double)g1;
    const double* gl = P.grad_lam + ((size_t)e1 * (NS + 1) + k1) * NS;
    double nn = 0.0;
#pragma unroll
    for (int d = 0; d < NS; ++d) nn += gl[d] * gl[d];
    nn = sqrt(nn);
#pragma unroll
    for (int d = 0; d < NS; ++d) G0[2 + d] = -gl[d] / nn;
#pragma unroll
    for (int i = 0; i <= NS; ++i)
#pragma unroll
      for (int d = 0; d <= NS; ++d) G0[2 + NS + i * (NS + 1) + d] = Pv[i][d];
  }
  __syncthreads();
  if (nbf > 0) {
    if (tid == 0) {
      int c = 0;
      for (int r = 0; r < m; ++r) {
        s_foff[r] = c;
        for (int f = 0; f < nbf; ++f)
          if ((int)FG[f * FGS + 1] == r) s_fl[c++] = f;
      }
      s_foff[m] = c;
    }
    __syncthreads();
    const long long gbase = P.bpt_off[tent];
    double* PN = PG;  // per-point outward normal (PCH x NS)
    if constexpr (MOM) {
      // Dirichlet terms from moments over the face points:
      //   A_ij += sum_q w [alpha c^2 v_i v_j + c v_i (s_j.n)],  b_i += sum_q w g (alpha c v_i - s_i.n)
      // (fields of the scaled basis; v = c vhat)
      const Tab& D = T;
      const int M2 = T.M2, M1 = T.M1;
      const int E2 = 2 * p - 1;
      double* NU = W1;                  // (NS+1) x M2: sum w m_b, sum w n_d m_b
      double* BV = NU + (NS + 1) * M2;  // (NS+1) x M1: sum w g m_k, sum w g n_d m_k
      double* POWT = POW;
      TaskRegs<kTaskSlots> RT;
      TaskRegs<kTaskSlots1> RB;
      load_tasks(T.task2, T.ntask2, RT);
      load_tasks(T.task1, T.ntask1, RB);
      for (int r = 0; r < m; ++r) {
        const int nf = s_foff[r + 1] - s_foff[r];
        if (nf == 0) continue;
        const double cr = gc[r], hr = gh[r];
        const int npts = nf * Q;
        for (int i = tid; i < (NS + 1) * (M2 + M1); i += blockDim.x) NU[i] = 0.0;
        // 3+1D: the geometric moments on the matrix cores, as the top moments of
        // the elements (tiles of (w L)^T R), face by face (the normal is constant
        // on a face: after its last chunk nu += C_f, nu_d += n_d C_f); chunks
        // then hold points of one face only
        bool fmt = false;
        if constexpr (NS == 3) fmt = Dp.mt_ntile > 0;
        const int fwave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int fnsl = (Dp.mt_ntile + 3) >> 2;
        unsigned ftex[kMomTileSlots];
        d4 facc[kMomTileSlots];
#pragma unroll
        for (int sl = 0; sl < kMomTileSlots; ++sl) {
          const int t = fwave + 4 * sl;
          ftex[sl] = (fmt && t < Dp.mt_ntile) ? (unsigned)Dp.mt_ex[t * 16 + (lane & 15)] : 0u;
          facc[sl] = d4{0.0, 0.0, 0.0, 0.0};
        }
        const int cpf = fmt ? (Q + PCH - 1) / PCH : 1;  // chunks per face (tile path)
        const int nchunk = fmt ? nf * cpf : (npts + PCH - 1) / PCH;
        __syncthreads();
        for (int cc = 0; cc < nchunk; ++cc) {
          const int f0 = fmt ? (cc / cpf) * Q + (cc % cpf) * PCH : cc * PCH;
          const int nc = fmt ? min(PCH, Q - (cc % cpf) * PCH) : min(PCH, npts - f0);
          const int nc4 = (nc + 3) & ~3;
          if (fmt)
            for (int pt = nc + tid; pt < nc4; pt += blockDim.x) {
              // points past the chunk up to a multiple of 4: weight 0, coordinates 0
              PW[pt] = 0.0;
              for (int v = 0; v <= NS; ++v) PV[pt * (NS + 1) + v] = 0.0;
            }
          for (int pt = tid; pt < nc; pt += blockDim.x) {
            const int fi = s_fl[s_foff[r] + (f0 + pt) / Q];
            const int q = (f0 + pt) % Q;
            const double* G0 = FG + fi * FGS;
            const double* lam = P.lam_ref + (size_t)q * (NS + 1);
            double y[NS + 1];
#pragma unroll
            for (int d = 0; d <= NS; ++d) y[d] = 0.0;
#pragma unroll
            for (int k = 0; k <= NS; ++k)
#pragma unroll
              for (int d = 0; d <= NS; ++d) y[d] += lam[k] * G0[2 + NS + k * (NS + 1) + d];
            const double w = P.w_ref[q] * G0[0];
            PW[pt] = w;
            PD[pt] = w * P.gD[gbase + (long long)fi * Q + q];
#pragma unroll
            for (int d = 0; d < NS; ++d) PN[pt * NS + d] = G0[2 + d];
            PV[pt * (NS + 1)] = cr * (y[NS] - tmid) / hr;
#pragma unroll
            for (int d = 0; d < NS; ++d) PV[pt * (NS + 1) + 1 + d] = (y[d] - XV[d]) / hr;
          }
          __syncthreads();
          for (int i = tid; i < (fmt ? nc4 : nc) * (NS + 1); i += blockDim.x) {
            const int pt = i / (NS + 1), v = i % (NS + 1);
            const double x = PV[pt * (NS + 1) + v];
            double a = 1.0;
            double* o = POWT + (pt * (NS + 1) + v) * E2;
            for (int ee = 0; ee < E2; ++ee) {
              o[ee] = a;
              a *= x;
            }
          }
          __syncthreads();
          if (fmt) {
            // geometric moments on the matrix cores (every wave runs wave 0's slot
            // count; a slot past the wave's tiles has exponents 0 and is not folded)
            for (int ks = 0; ks < (nc4 >> 2); ++ks) {
              const int pt = ks * 4 + (lane >> 4);
              const double* pw = POWT + pt * (NS + 1) * E2;
              const double w = PW[pt];
#pragma unroll
              for (int sl = 0; sl < kMomTileSlots; ++sl) {
                if (sl < fnsl) {
                  const unsigned ex = ftex[sl];
                  const double a = w * (pw[ex & 31u] * pw[E2 + ((ex >> 5) & 31u)]);
                  const double b = pw[2 * E2 + ((ex >> 10) & 31u)] * pw[3 * E2 + ((ex >> 15) & 31u)];
                  facc[sl] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, facc[sl], 0, 0, 0);
                }
              }
            }
          }
          // geometric moments (w, w n_d) over the moment monomials
#pragma unroll
          for (int sl = 0; sl < kTaskSlots; ++sl) {
            if (fmt) break;
            if (tid + sl * (int)blockDim.x >= T.ntask2) break;
            const unsigned w0 = RT.w0[sl];
            int e[NS];
#pragma unroll
            for (int v = 0; v < NS; ++v) e[v] = task_exp(w0, v);
            const int d0 = task_exp(w0, 3);
            double a0[4], ad[4][NS];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              a0[c] = 0.0;
#pragma unroll
              for (int d = 0; d < NS; ++d) ad[c][d] = 0.0;
            }
#pragma unroll 1
            for (int pt = 0; pt < nc; ++pt) {
              const double* pw = POWT + pt * (NS + 1) * E2;
              double pre = pw[e[0]];
#pragma unroll
              for (int v = 1; v < NS; ++v) pre *= pw[v * E2 + e[v]];
              const double z = E2 > 1 ? pw[NS * E2 + 1] : 0.0;
              double mv = pre * pw[NS * E2 + d0];
              const double w = PW[pt];
              double nn[NS];
#pragma unroll
              for (int d = 0; d < NS; ++d) nn[d] = w * PN[pt * NS + d];
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                a0[c] += w * mv;
#pragma unroll
                for (int d = 0; d < NS; ++d) ad[c][d] += nn[d] * mv;
                mv *= z;
              }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const int b = task_idx(RT, sl, c);
              if (b < 0) continue;
              NU[b] += a0[c];
#pragma unroll
              for (int d = 0; d < NS; ++d) NU[(1 + d) * M2 + b] += ad[c][d];
            }
          }
          // data moments (w g, w g n_d) over the monomials of degree <= p-1 (the
          // first M1 monomials; runs starting beyond them are skipped)
#pragma unroll
          for (int sl = 0; sl < kTaskSlots1; ++sl) {
            if (tid + sl * (int)blockDim.x >= T.ntask1) break;
            if (task_idx(RB, sl, 0) >= M1) continue;
            const unsigned w0 = RB.w0[sl];
            int e[NS];
#pragma unroll
            for (int v = 0; v < NS; ++v) e[v] = task_exp(w0, v);
            const int d0 = task_exp(w0, 3);
            double g0[4], gd[4][NS];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              g0[c] = 0.0;
#pragma unroll
              for (int d = 0; d < NS; ++d) gd[c][d] = 0.0;
            }
#pragma unroll 1
            for (int pt = 0; pt < nc; ++pt) {
              const double* pw = POWT + pt * (NS + 1) * E2;
              double pre = pw[e[0]];
#pragma unroll
              for (int v = 1; v < NS; ++v) pre *= pw[v * E2 + e[v]];
              const double z = E2 > 1 ? pw[NS * E2 + 1] : 0.0;
              double mv = pre * pw[NS * E2 + d0];
              const double g = PD[pt];
              double nn[NS];
#pragma unroll
              for (int d = 0; d < NS; ++d) nn[d] = g * PN[pt * NS + d];
#pragma unroll
              for (int c = 0; c < 4; ++c) {
                g0[c] += g * mv;
#pragma unroll
                for (int d = 0; d < NS; ++d) gd[c][d] += nn[d] * mv;
                mv *= z;
              }
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const int k = task_idx(RB, sl, c);
              if (k < 0 || k >= M1) continue;
              BV[k] += g0[c];
#pragma unroll
              for (int d = 0; d < NS; ++d) BV[(1 + d) * M1 + k] += gd[c][d];
            }
          }
          __syncthreads();
          if (fmt && cc % cpf == cpf - 1) {
            // the face's tiles into the moments (each moment index belongs to one
            // tile entry: no two lanes or waves write the same word)
            const double* G0 = FG + s_fl[s_foff[r] + cc / cpf] * FGS;
            double nrm[NS];
#pragma unroll
            for (int d = 0; d < NS; ++d) nrm[d] = G0[2 + d];
#pragma unroll
            for (int sl = 0; sl < kMomTileSlots; ++sl) {
              const int t = fwave + 4 * sl;
              if (t < Dp.mt_ntile) {
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4) {
                  const int b = Dp.mt_map[t * 256 + ((lane >> 4) + 4 * e4) * 16 + (lane & 15)];
                  if (b >= 0) {
                    const double c = facc[sl][e4];
                    NU[b] += c;
#pragma unroll
                    for (int d = 0; d < NS; ++d) NU[(1 + d) * M2 + b] += nrm[d] * c;
                  }
                }
              }
              facc[sl] = d4{0.0, 0.0, 0.0, 0.0};
            }
            __syncthreads();
          }
        }
        for (int i = tid; i < NW; i += blockDim.x) {
          double b = 0.0;
          for (int a = 0; a <= NS; ++a) {
            const int row = i * (NS + 1) + a;
            const double sc = a == 0 ? P.alpha * cr : -1.0;
            for (int e = D.fo_ptr[row]; e < D.fo_ptr[row + 1]; ++e)
              b += D.fo_coef[e] * sc * BV[a * M1 + D.fo_idx[e]];
          }
          AT[(long long)(r * NW + i) * lda + S] += b;
        }
        __syncthreads();
        moment_gram_block<NS>(T.fo_ptr, T.fo_idx, T.fo_coef, T.K2, M1, M2, NW, NU, BV,
                              (long long)(L.off_fg - L.off_W1) - (long long)(NS + 1) * M2, cr, P.alpha, true, AT, lda,
                              r * NW);
      }
    } else {
    for (int r = 0; r < m; ++r) {
      const int nf = s_foff[r + 1] - s_foff[r];
      if (nf == 0) continue;
      const double cr = gc[r], hr = gh[r];
      const int npts = nf * Q;
      for (int f0 = 0; f0 < npts; f0 += PCH) {
        const int nc = min(PCH, npts - f0);
        for (int pt = tid; pt < PCH; pt += blockDim.x) {
          double y[NS + 1];
#pragma unroll
          for (int d = 0; d < NS; ++d) y[d] = XV[d];
          y[NS] = tmid;
          double w = 0.0, g = 0.0;
          if (pt < nc) {
            const int fi = s_fl[s_foff[r] + (f0 + pt) / Q];
            const int q = (f0 + pt) % Q;
            const double* G0 = FG + fi * FGS;
            const double* lam = P.lam_ref + (size_t)q * (NS + 1);
#pragma unroll
            for (int d = 0; d <= NS; ++d) y[d] = 0.0;
#pragma unroll
            for (int k = 0; k <= NS; ++k)
#pragma unroll
              for (int d = 0; d <= NS; ++d) y[d] += lam[k] * G0[2 + NS + k * (NS + 1) + d];
            w = P.w_ref[q] * G0[0];
            g = P.gD[gbase + (long long)fi * Q + q];
#pragma unroll
            for (int d = 0; d < NS; ++d) PN[pt * NS + d] = G0[2 + d];
          }
          PV[pt * (NS + 1)] = cr * (y[NS] - tmid) / hr;
#pragma unroll
          for (int d = 0; d < NS; ++d) PV[pt * (NS + 1) + 1 + d] = (y[d] - XV[d]) / hr;
          PW[pt] = w;
          PD[pt] = g;
        }
        __syncthreads();
        monomials<NS>(T, T.M1, p, PV, POW, MT, PCH, PCH);
        __syncthreads();
        for (int i = tid; i < PCH * NW; i += blockDim.x) {
          const int pt = i % PCH, j = i / PCH;
          const double w = PW[pt], sw = sqrt(w), g = PD[pt];
          double fl[NS + 1], uu;
          eval_j<NS, false>(T, j, MT, PCH, pt, fl, &uu);
          const double v = cr * fl[0];
          double sn = 0.0;
          if (pt < nc)
#pragma unroll
            for (int d = 0; d < NS; ++d) sn += fl[1 + d] * PN[pt * NS + d];
          F1[pt * NWP + j] = sw * v;
          F1[(PCH + pt) * NWP + j] = sw * (P.alpha * v + sn);
          F1[(2 * PCH + pt) * NWP + j] = w * g * (P.alpha * v - sn);
        }
        __syncthreads();
        for (int idx = tid; idx < NW * NW; idx += blockDim.x) {
          const int ii = idx / NW, jj = idx % NW;
          double acc = 0.0;
          for (int k = 0; k < nc; ++k) acc += F1[k * NWP + ii] * F1[(PCH + k) * NWP + jj];
          AT[(long long)(r * NW + ii) * lda + r * NW + jj] += acc;
        }
        for (int j = tid; j < NW; j += blockDim.x) {
          double acc = 0.0;
          for (int k = 0; k < nc; ++k) acc += F1[(2 * PCH + k) * NWP + j];
          AT[(long long)(r * NW + j) * lda + S] += acc;
        }
        __syncthreads();
      }
    }
    }  // quadrature faces
  }
  // 3b. speed interfaces, then Neumann faces (eq. 4.1, T^N), one face at a time
  //     (chunks of PCI points; in moment mode the monomials sit in W1 behind the
  //     face values)
  double* MTI = MOM ? W1 + 4 * PCI * NWP : MT;
  const int nnf = P.vn_ptr[V + 1] - P.vn_ptr[V];
  for (int f = 0; f < nif + nnf; ++f) {
    const bool dir = f >= nif;  // a Neumann face: one side, data g_N
    int e1, k1, e2 = -1;
    if (dir) {
      e1 = P.vn[2 * (P.vn_ptr[V] + f - nif)];
      k1 = P.vn[2 * (P.vn_ptr[V] + f - nif) + 1];
    } else {
      const int* q4 = P.vi + 4 * (P.vi_ptr[V] + f);
      e1 = q4[0];
      k1 = q4[1];
      e2 = q4[2];
    }
    if (tid == 0) {
      // space-time simplex (X_V, tb), (X_V, tt), (X_W, tau_W) for W in facet \ {V}
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
      int g1 = 0, g2 = 0;
      for (int i = 0; i < npatch; ++i) {
        const int e = (int)EL[i * ELS + El<NS>::E];
        if (e == e1) g1 = (int)EL[i * ELS + El<NS>::GRP];
        if (e == e2) g2 = (int)EL[i * ELS + El<NS>::GRP];
      }
      s_piv = g1 * kMaxGroups + g2;  // (both below kMaxGroups)
    }
    __syncthreads();
    const double meas = fsc[0];
    double nrm[NS];
    for (int d = 0; d < NS; ++d) nrm[d] = fsc[1 + d];
    const int ga = s_piv / kMaxGroups, gb = s_piv % kMaxGroups;
    // g_N of a Neumann face: after the tent's Dirichlet faces in the boundary data
    const long long goff = P.bpt_off[tent] + (long long)(nbf + f - nif) * Q;
    for (int q0 = 0; q0 < Q; q0 += PCI) {
      const int nc = min(PCI, Q - q0);
      const int nside = dir ? 1 : 2;
      for (int side = 0; side < nside; ++side) {
        const int r = side == 0 ? ga : gb;
        const double cr = gc[r], hr = gh[r];
        for (int pt = tid; pt < PCI; pt += blockDim.x) {
          double y[NS + 1];
          for (int d = 0; d < NS; ++d) y[d] = XV[d];
          y[NS] = tmid;
          double w = 0.0, g = 0.0;
          if (pt < nc) {
            const int q = q0 + pt;
            const double* lam = P.lam_ref + (size_t)q * (NS + 1);
            for (int d = 0; d <= NS; ++d) y[d] = 0.0;
            for (int k = 0; k <= NS; ++k)
              for (int d = 0; d <= NS; ++d) y[d] += lam[k] * fsc[4 + k * (NS + 1) + d];
            w = P.w_ref[q] * meas;
            if (dir) g = P.gD[goff + q];
          }
          PV[pt * (NS + 1)] = cr * (y[NS] - tmid) / hr;
          for (int d = 0; d < NS; ++d) PV[pt * (NS + 1) + 1 + d] = (y[d] - XV[d]) / hr;
          PW[pt] = w;
          PD[pt] = g;
        }
        __syncthreads();
        monomials<NS>(T, T.M1, p, PV, POW, MTI, PCI, PCI);
        __syncthreads();
        for (int i = tid; i < PCI * NW; i += blockDim.x) {
          const int pt = i % PCI, j = i / PCI;
          const double w = PW[pt], sw = sqrt(w), g = PD[pt];
          double fl[NS + 1], uu;
          eval_j<NS, false>(T, j, MTI, PCI, pt, fl, &uu);
          const double v = cr * fl[0];
          double sn = 0.0;
          for (int d = 0; d < NS; ++d) sn += fl[1 + d] * nrm[d];
          if (dir) {
            // test tau_i.n, trial v_j + beta sigma_j.n; data g_N (beta tau_i.n - w_i)
            F1[pt * NWP + j] = sw * sn;
            F1[(PCI + pt) * NWP + j] = sw * (v + P.beta * sn);
            F1[(2 * PCI + pt) * NWP + j] = w * g * (P.beta * sn - v);
          } else {
            F1[((2 * side) * PCI + pt) * NWP + j] = sw * v;
            F1[((2 * side + 1) * PCI + pt) * NWP + j] = sw * sn;
          }
        }
        __syncthreads();
      }
      if (dir) {
        for (int idx = tid; idx < NW * NW; idx += blockDim.x) {
          const int ii = idx / NW, jj = idx % NW;
          double acc = 0.0;
          for (int k = 0; k < nc; ++k) acc += F1[k * NWP + ii] * F1[(PCI + k) * NWP + jj];
          AT[(long long)(ga * NW + ii) * lda + ga * NW + jj] += acc;
        }
        for (int j = tid; j < NW; j += blockDim.x) {
          double acc = 0.0;
          for (int k = 0; k < nc; ++k) acc += F1[(2 * PCI + k) * NWP + j];
          AT[(long long)(ga * NW + j) * lda + S] += acc;
        }
      } else {
        // test in group b (sign sb), trial in group a (sign sa):
        // w_i (alpha sa sb v_j + sb/2 s_j.n) + (tau_i.n)(sb/2 v_j + beta sa sb s_j.n)
        for (int blk = 0; blk < 4; ++blk) {
          const int sa_i = blk / 2, sb_i = blk % 2;
          const double sa = sa_i ? -1.0 : 1.0, sb = sb_i ? -1.0 : 1.0;
          const int gA = sa_i ? gb : ga, gB = sb_i ? gb : ga;
          const double* Va = F1 + (2 * sa_i) * PCI * NWP;
          const double* Na = F1 + (2 * sa_i + 1) * PCI * NWP;
          const double* Vb = F1 + (2 * sb_i) * PCI * NWP;
          const double* Nb = F1 + (2 * sb_i + 1) * PCI * NWP;
          for (int idx = tid; idx < NW * NW; idx += blockDim.x) {
            const int ii = idx / NW, jj = idx % NW;
            double acc = 0.0;
            for (int k = 0; k < nc; ++k) {
              const double va = Va[k * NWP + jj], na = Na[k * NWP + jj];
              acc += Vb[k * NWP + ii] * (P.alpha * sa * sb * va + 0.5 * sb * na) +
                     Nb[k * NWP + ii] * (0.5 * sb * va + P.beta * sa * sb * na);
            }
            AT[(long long)(gB * NW + ii) * lda + gA * NW + jj] += acc;
          }
        }
      }
      __syncthreads();
    }
  }

  // ---- 4. local solve ------------------------------------------------------------------
  if constexpr (MIXED) {
    for (long long i = tid; i < (long long)S * lda; i += blockDim.x) A[i] += AF[i];
    __syncthreads();
  }
  if (!MIXED || !use32) {
    // FP64 system: LU, then back substitution
    bool ok;
    if (S <= 32 && L.A_in_lds) {
      bool w_ok = true;
      if (wave == 0) w_ok = wave_lu_regs<32>(A, (int)lda, S, xs);
      if (wave == 0 && lane == 0 && !w_ok) s_err = kStatSingular;
      __syncthreads();
      ok = s_err == 0;
    } else {
      // the blocked LU is compiled into the 3+1D kernels only (2+1D systems
      // stay in LDS in the workloads here, and the extra registers would
      // halve the occupancy of the 2+1D kernels)
      bool done = false;
      if constexpr (NS == 3) {
        if (!L.A_in_lds && L.lu_nb > 0) {
          ok = panel_lu_solve(A, lda, S, L.lu_nb, xs, lds + L.off_pow);
          __syncthreads();
          done = true;
        }
      }
      if (!done) {
        ok = block_lu_solve(A, lda, S, xs, &s_piv);
        __syncthreads();
      }
    }
    if (!ok) {
      if (tid == 0) atomicOr(P.status, kStatSingular);
      return;
    }
    break;
  }
  if constexpr (MIXED) {
    // FP32-assembled system: factor once, solve, refine with the FP64 residual
    // r = b - (Psi64^T Psi64) x - F x, evaluated matrix-free over the top points
    for (int i = tid; i < S; i += blockDim.x) bvec[i] = A[(long long)i * lda + S];
    __syncthreads();
    const bool fac_ok = block_lu_factor(A, lda, S);
    __syncthreads();
    if (!fac_ok) {
      use32 = false;
      continue;
    }
    for (int i = tid; i < S; i += blockDim.x) xs[i] = bvec[i];
    __syncthreads();
    block_lu_apply(A, lda, S, xs);
    __syncthreads();
    double dn_prev = INFINITY;
    if (tid == 0) s_conv = 0;
    for (int it = 0; it < kIRMax; ++it) {
      // residual: b - F x
      for (int i = tid; i < S; i += blockDim.x) {
        double sacc = 0.0;
        for (int j = 0; j < S; ++j) sacc += AF[(long long)i * lda + j] * xs[j];
        rvec[i] = bvec[i] - sacc;
      }
      __syncthreads();
      // ... - Psi64^T (Psi64 x), group by group, chunk by chunk
      for (int r = 0; r < m; ++r) {
        const double cr = gc[r], hr = gh[r];
        const int npts = (s_goff[r + 1] - s_goff[r]) * Q;
        for (int f0 = 0; f0 < npts; f0 += PCH) {
          const int nc = min(PCH, npts - f0);
          for (int pt = tid; pt < PCH; pt += blockDim.x) {
            double xt[NS], g[NS];
            double phi = tmid, w = 0.0, sD = 0.0;
            for (int d = 0; d < NS; ++d) {
              xt[d] = XV[d];
              g[d] = 0.0;
            }
            if (pt < nc) {
              const int f = f0 + pt;
              const double* R = EL + s_gel[s_goff[r] + f / Q] * ELS;
              const int q = f % Q;
              const int lV = (int)R[El<NS>::LV];
              const double* lam = P.lam_ref + (size_t)q * (NS + 1);
              phi = 0.0;
              for (int d = 0; d < NS; ++d) xt[d] = 0.0;
              for (int k = 0; k <= NS; ++k) {
                phi += lam[k] * R[El<NS>::TAU + k];
                for (int d = 0; d < NS; ++d) xt[d] += lam[k] * R[El<NS>::X + k * NS + d];
              }
              phi += lam[lV] * dt;
              w = P.w_ref[q] * R[El<NS>::DET];
              double gn2 = 0.0;
              for (int d = 0; d < NS; ++d) {
                g[d] = R[El<NS>::GNEW + d];
                gn2 += g[d] * g[d];
              }
              sD = 1.0 / (cr * cr) - gn2;
            }
            PV[pt * (NS + 1)] = cr * (phi - tmid) / hr;
            for (int d = 0; d < NS; ++d) {
              PV[pt * (NS + 1) + 1 + d] = (xt[d] - XV[d]) / hr;
              PG[pt * NS + d] = g[d];
            }
            PW[pt] = w;
            PS[pt] = sD;
          }
          __syncthreads();
          monomials<NS>(T, T.M1, p, PV, POW, MT, PCH, PCH);
          __syncthreads();
          for (int i = tid; i < PCH * NW; i += blockDim.x) {
            const int pt = i % PCH, j = i / PCH;
            const double w = PW[pt];
            const double sw = sqrt(w), swD = sqrt(w * PS[pt]);
            double f[NS + 1], uu;
            eval_j<NS, false>(T, j, MT, PCH, pt, f, &uu);
            const double v = cr * f[0];
            double* row = PSI + (size_t)pt * (NS + 1) * NWP + j;
            row[0] = swD * v;
            for (int d = 0; d < NS; ++d) row[(1 + d) * NWP] = sw * (f[1 + d] - PG[pt * NS + d] * v);
          }
          __syncthreads();
          double* yv = RB;  // Psi64 x, one value per row of the chunk
          for (int row = tid; row < nc * (NS + 1); row += blockDim.x) {
            double sacc = 0.0;
            for (int j = 0; j < NW; ++j) sacc += PSI[(size_t)row * NWP + j] * xs[r * NW + j];
            yv[row] = sacc;
          }
          __syncthreads();
          for (int j = tid; j < NW; j += blockDim.x) {
            double sacc = 0.0;
            for (int row = 0; row < nc * (NS + 1); ++row) sacc += PSI[(size_t)row * NWP + j] * yv[row];
            rvec[r * NW + j] -= sacc;
          }
          __syncthreads();
        }
      }
      block_lu_apply(A, lda, S, rvec);
      // correction norms (max over the block)
      double dloc = 0.0, xloc = 0.0;
      for (int i = tid; i < S; i += blockDim.x) {
        const double xn = xs[i] + rvec[i];
        dloc = fmax(dloc, fabs(rvec[i]));
        xloc = fmax(xloc, fabs(xn));
        xs[i] = xn;
      }
      for (int off = 32; off > 0; off >>= 1) {
        dloc = fmax(dloc, __shfl_xor(dloc, off, 64));
        xloc = fmax(xloc, __shfl_xor(xloc, off, 64));
      }
      if (lane == 0) {
        s_red[2 * wave] = dloc;
        s_red[2 * wave + 1] = xloc;
      }
      __syncthreads();
      double dn = 0.0, xn = 0.0;
      for (int w = 0; w < (int)blockDim.x / 64; ++w) {
        dn = fmax(dn, s_red[2 * w]);
        xn = fmax(xn, s_red[2 * w + 1]);
      }
      ir_steps = it + 1;
      const bool done = dn <= 1e-12 * xn;
      const bool stalled = !done && dn > 0.5 * dn_prev;
      dn_prev = dn;
      __syncthreads();
      if (done || stalled) {
        if (tid == 0) s_conv = dn <= 1e-10 * xn ? 1 : 0;
        break;
      }
    }
    __syncthreads();
    if (s_conv) break;
    use32 = false;  // refinement did not reach FP64 accuracy: FP64 Gram for this tent
  }
  }  // attempts
  if (MIXED && tid == 0 && P.ir_steps) P.ir_steps[tent] = ir_steps + (use32 ? 0 : 1000);
  if (tid < m) {
    if (R2) {
      a0[tid] = xs[S0 + tid];
    } else {
      double s = r0[tid];
      for (int j = 0; j < NW; ++j) s -= A0[tid * NWP + j] * xs[tid * NW + j];
      a0[tid] = P.recover_U ? s / A00[tid] : 0.0;
    }
  }
  __syncthreads();

  // ---- 5. indicator: energy of the jump between the solution and the incoming
  //         trace on the bottom facets, 1/2 B_phi_old(u - u_b, u - u_b)
  // Sections 5 and 6 evaluate the solution one point per thread: the monomials of
  // a point come from the runs of the degree-p table (a shared prefix times
  // consecutive powers of the last variable), the coefficients cm are read by all
  // threads at the same address.
  double* cm = W1;  // (NS+2) x M: coefficients of v, sigma, U on the monomials, contracted with x
  // the monomial runs of degree p, staged behind cm (read by all threads at once)
  int* runs = reinterpret_cast<int*>(W1 + (((NS + 2) * T.M + 3) & ~3));
  for (int i = tid; i < T.ntask1 * kTaskInts; i += blockDim.x) runs[i] = T.task1[i];
  const bool want_eta = P.indicator || !P.write_back || (P.eta_tol > 0.0 && p < P.pmax);
  bool wb_done = false;  // the top values were formed with the indicator (into TMP)
  if (want_eta) {
    double eta_loc = 0.0;
    for (int r = 0; r < m; ++r) {
      const double cr = gc[r], hr = gh[r];
      const double ic2 = 1.0 / (cr * cr);
      const int npts = (s_goff[r + 1] - s_goff[r]) * Q;
      bool ev_mt = false;
      if constexpr (NS == 3) ev_mt = Dp.ev_nl > 0 && (long long)(L.off_fg - L.off_W1) >= ev_doubles(p, Dp.ev_nl);
      if constexpr (NS == 3) {
        // One speed group, a write-back to follow and room for it: the top values
        // are formed in the same pass (the products Y of the evaluation do not
        // depend on the time coordinate) into the workgroup's global slot, which
        // the solved system no longer needs, and copied to the stored values once
        // the tent is accepted (the stored values stay the incoming ones until
        // then, as a solve at a higher degree needs them).
        constexpr int kFuseSteps = 9;  // tile-0 steps of the one-pass evaluation (p <= 7)
        const bool fuse = ev_mt && m == 1 && P.write_back && !L.A_in_lds && Dp.ev_nks[0] <= kFuseSteps &&
                          (long long)npts * (NS + 2) <= P.work_stride &&
                          (long long)(L.off_fg - L.off_W1) >= ev_doubles(p, Dp.ev_nl) + 4LL * 16 * (p + 1) + 4 * 16 * 5;
        if (fuse) {
          const int nl = Dp.ev_nl, nat = Dp.ev_nat, nA16 = 16 * nat, ldb = ev_ldb(nl), P1 = p + 1;
          double* CMd = W1;
          double* PWW = W1 + (long long)(NS + 2) * nA16 * ldb;
          double* SVW = PWW + 4 * 16 * 5 * P1;  // per wave and point: incoming v, sigma and the weight
          int* EXs = reinterpret_cast<int*>(SVW + 4 * 16 * 5);
          double* TMP = A;  // (NS+2) x npts top values
          __syncthreads();
          for (int i = tid; i < nl; i += blockDim.x) EXs[i] = Dp.ev_ex[i];
          build_cm_dense<NS>(T, Dp, xs + r * NW, hr, CMd, nA16, ldb);
          double* pwv = PWW + wave * 16 * 5 * P1;
          double* svw = SVW + wave * 16 * 5;
          // lane l < 16 holds the reference coordinates, incoming values and
          // weight of its point of the next block, loaded while the current
          // block is evaluated
          double lamn[NS + 1], stn[NS + 2];
          auto load_lam = [&](int blk) {
            const int f = min(blk + wave * 16 + lane, npts - 1);
            const double* R = EL + s_gel[s_goff[r] + f / Q] * ELS;
            const int q = f % Q;
            const double* st = P.state + (size_t)(int)R[El<NS>::E] * (NS + 2) * Q;
#pragma unroll
            for (int k = 0; k <= NS; ++k) lamn[k] = gload(P.lam_ref + (size_t)q * (NS + 1) + k);
#pragma unroll
            for (int c = 0; c <= NS; ++c) stn[c] = gload(st + c * Q + q);
            stn[NS + 1] = gload(P.w_ref + q) * R[El<NS>::DET];
          };
          if (lane < 16) load_lam(0);
          for (int blk = 0; blk < npts; blk += 64) {
            if (lane < 16) {
              // rows: th at the bottom, xh_1..xh_n, th at the top
              const int f = min(blk + wave * 16 + lane, npts - 1);
              const double* R = EL + s_gel[s_goff[r] + f / Q] * ELS;
              const int lV = (int)R[El<NS>::LV];
              double var[NS + 2], pho = 0.0;
              for (int d = 1; d <= NS; ++d) var[d] = 0.0;
              for (int k = 0; k <= NS; ++k) {
                pho += lamn[k] * R[El<NS>::TAU + k];
                for (int d = 0; d < NS; ++d) var[1 + d] += lamn[k] * R[El<NS>::X + k * NS + d];
              }
              double lv = lamn[0];
#pragma unroll
              for (int k = 1; k <= NS; ++k)
                if (k == lV) lv = lamn[k];
              var[0] = cr * (pho - tmid) / hr;
              var[NS + 1] = cr * (pho + lv * dt - tmid) / hr;
              for (int d = 0; d < NS; ++d) var[1 + d] = (var[1 + d] - XV[d]) / hr;
              for (int v = 0; v <= NS + 1; ++v) {
                double a = 1.0;
                for (int e = 0; e < P1; ++e) {
                  pwv[(lane * 5 + v) * P1 + e] = a;
                  a *= var[v];
                }
              }
#pragma unroll
              for (int c = 0; c < NS + 2; ++c) svw[lane * 5 + c] = stn[c];
              if (blk + 64 < npts) load_lam(blk + 64);
            }
            wave_sync();
            double valb[NS + 1][4], valt[NS + 2][4];
            eval16_mfma2<NS + 2, NS + 1, NS + 1, kFuseSteps>(CMd, nA16, ldb, nl, nat, Dp.ev_nks, Dp.ev_nkv, EXs, pwv,
                                                              P1, valb, valt);
            if ((lane & 15) == 0) {
#pragma unroll
              for (int rr = 0; rr < 4; ++rr) {
                const int f = blk + wave * 16 + (lane >> 4) + 4 * rr;
                if (f < npts) {
                  const double* R = EL + s_gel[s_goff[r] + f / Q] * ELS;
                  const double* sv = svw + ((lane >> 4) + 4 * rr) * 5;
                  const double dv = cr * valb[0][rr] - sv[0];
                  double ds2 = 0.0, dsg = 0.0;
                  for (int d = 0; d < NS; ++d) {
                    const double ds = valb[1 + d][rr] - sv[1 + d];
                    ds2 += ds * ds;
                    dsg += ds * R[El<NS>::GOLD + d];
                  }
                  eta_loc += 0.5 * sv[NS + 1] * (ic2 * dv * dv + ds2 - 2.0 * dv * dsg);
                  TMP[f] = cr * valt[0][rr];
#pragma unroll
                  for (int d = 0; d < NS; ++d) TMP[(long long)(1 + d) * npts + f] = valt[1 + d][rr];
                  TMP[(long long)(NS + 1) * npts + f] = a0[r] + valt[NS + 1][rr];
                  bool fin = true;
#pragma unroll
                  for (int c = 0; c < NS + 2; ++c) fin = fin && isfinite(valt[c][rr]);
                  if (!fin) atomicOr(P.status, kStatNan);
                }
              }
            }
            wave_sync();
          }
          wb_done = true;
          continue;
        }
        if (ev_mt) {
          // fields at the bottom points on the matrix cores, 16 points per wave
          const int nl = Dp.ev_nl, nat = Dp.ev_nat, nA16 = 16 * nat, ldb = ev_ldb(nl), P1 = p + 1;
          double* CMd = W1;
          double* PWW = W1 + (long long)(NS + 2) * nA16 * ldb;
          int* EXs = reinterpret_cast<int*>(PWW + 4 * 16 * 4 * P1);
          __syncthreads();
          for (int i = tid; i < nl; i += blockDim.x) EXs[i] = Dp.ev_ex[i];
          build_cm_dense<NS>(T, Dp, xs + r * NW, hr, CMd, nA16, ldb);
          double* pwv = PWW + wave * 16 * 4 * P1;
          // lane l < 16 holds the reference coordinates of its point of the next
          // block, loaded while the current block is evaluated
          double lamn[NS + 1];
          auto load_lam = [&](int blk) {
            const int f = min(blk + wave * 16 + lane, npts - 1);
#pragma unroll
            for (int k = 0; k <= NS; ++k) lamn[k] = gload(P.lam_ref + (size_t)(f % Q) * (NS + 1) + k);
          };
          if (lane < 16) load_lam(0);
          for (int blk = 0; blk < npts; blk += 64) {
            if (lane < 16) {
              const int f = min(blk + wave * 16 + lane, npts - 1);
              const double* R = EL + s_gel[s_goff[r] + f / Q] * ELS;
              double var[NS + 1], phi = 0.0;
              for (int d = 1; d <= NS; ++d) var[d] = 0.0;
              for (int k = 0; k <= NS; ++k) {
                phi += lamn[k] * R[El<NS>::TAU + k];
                for (int d = 0; d < NS; ++d) var[1 + d] += lamn[k] * R[El<NS>::X + k * NS + d];
              }
              var[0] = cr * (phi - tmid) / hr;
              for (int d = 0; d < NS; ++d) var[1 + d] = (var[1 + d] - XV[d]) / hr;
              for (int v = 0; v <= NS; ++v) {
                double a = 1.0;
                for (int e = 0; e < P1; ++e) {
                  pwv[(lane * 4 + v) * P1 + e] = a;
                  a *= var[v];
                }
              }
              if (blk + 64 < npts) load_lam(blk + 64);
            }
            wave_sync();
            // the incoming values and weights of the four points of this lane's
            // row, loaded before the evaluation
            double stv[4][NS + 1], wq[4];
            if ((lane & 15) == 0) {
#pragma unroll
              for (int rr = 0; rr < 4; ++rr) {
                const int f = min(blk + wave * 16 + (lane >> 4) + 4 * rr, npts - 1);
                const double* R = EL + s_gel[s_goff[r] + f / Q] * ELS;
                const int q = f % Q;
                const double* st = P.state + (size_t)(int)R[El<NS>::E] * (NS + 2) * Q;
#pragma unroll
                for (int c = 0; c <= NS; ++c) stv[rr][c] = gload(st + c * Q + q);
                wq[rr] = gload(P.w_ref + q) * R[El<NS>::DET];
              }
            }
            double val[NS + 1][4];
            eval16_mfma<NS + 1, NS + 1>(CMd, nA16, ldb, nl, nat, Dp.ev_nks, Dp.ev_nkv, EXs, pwv, P1, val);
            if ((lane & 15) == 0) {
#pragma unroll
              for (int rr = 0; rr < 4; ++rr) {
                const int f = blk + wave * 16 + (lane >> 4) + 4 * rr;
                if (f < npts) {
                  const double* R = EL + s_gel[s_goff[r] + f / Q] * ELS;
                  const double dv = cr * val[0][rr] - stv[rr][0];
                  double ds2 = 0.0, dsg = 0.0;
                  for (int d = 0; d < NS; ++d) {
                    const double ds = val[1 + d][rr] - stv[rr][1 + d];
                    ds2 += ds * ds;
                    dsg += ds * R[El<NS>::GOLD + d];
                  }
                  eta_loc += 0.5 * wq[rr] * (ic2 * dv * dv + ds2 - 2.0 * dv * dsg);
                }
              }
            }
            wave_sync();
          }
          continue;
        }
      }
      __syncthreads();
      for (int row = tid; row < (NS + 1) * T.M; row += blockDim.x) {
        double acc = 0.0;
        for (int e = T.tr_ptr[row]; e < T.tr_ptr[row + 1]; ++e) acc += T.tr_coef[e] * xs[r * NW + T.tr_j[e]];
        cm[row] = acc;
      }
      __syncthreads();
      for (int f = tid; f < npts; f += blockDim.x) {
        const double* R = EL + s_gel[s_goff[r] + f / Q] * ELS;
        const int q = f % Q;
        const double* lam = P.lam_ref + (size_t)q * (NS + 1);
        double xt[NS], phi = 0.0;
        for (int d = 0; d < NS; ++d) xt[d] = 0.0;
        for (int k = 0; k <= NS; ++k) {
          phi += lam[k] * R[El<NS>::TAU + k];
          for (int d = 0; d < NS; ++d) xt[d] += lam[k] * R[El<NS>::X + k * NS + d];
        }
        double var[NS + 1];
        var[0] = cr * (phi - tmid) / hr;
        for (int d = 0; d < NS; ++d) var[1 + d] = (xt[d] - XV[d]) / hr;
        double val[NS + 1];
#pragma unroll
        for (int c = 0; c <= NS; ++c) val[c] = 0.0;
        eval_runs<NS, false>(T, runs, var, cm, val);
        const int e = (int)R[El<NS>::E];
        const double w = P.w_ref[q] * R[El<NS>::DET];
        const double* st = P.state + (size_t)e * (NS + 2) * Q;
        const double dv = cr * val[0] - st[q];
        double ds2 = 0.0, dsg = 0.0;
        for (int d = 0; d < NS; ++d) {
          const double ds = val[1 + d] - st[(1 + d) * Q + q];
          ds2 += ds * ds;
          dsg += ds * R[El<NS>::GOLD + d];
        }
        eta_loc += 0.5 * w * (ic2 * dv * dv + ds2 - 2.0 * dv * dsg);
      }
    }
    // deterministic workgroup sum
    for (int off = 32; off > 0; off >>= 1) eta_loc += __shfl_xor(eta_loc, off, 64);
    __syncthreads();
    if (lane == 0) s_red[wave] = eta_loc;
    __syncthreads();
    double eta = 0.0;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) eta += s_red[w];
    const bool redo = P.eta_tol > 0.0 && p < P.pmax && eta > P.eta_tol;
    __syncthreads();
    if (redo) continue;
    if (tid == 0 && P.dissip) P.dissip[tent] = eta;
    if (tid == 0 && P.p_used) P.p_used[tent] = (signed char)p;
    if (!P.write_back) return;
    if (wb_done) {
      // the accepted tent's top values (one group) from the global slot
      const int npts = (s_goff[1] - s_goff[0]) * Q;
      const double* TMP = A;
      __threadfence_block();
      for (int f = tid; f < npts; f += blockDim.x) {
        const double* R = EL + s_gel[s_goff[0] + f / Q] * ELS;
        const int q = f % Q;
        double* st = P.state + (size_t)(int)R[El<NS>::E] * (NS + 2) * Q;
#pragma unroll
        for (int c = 0; c < NS + 2; ++c) st[(long long)c * Q + q] = TMP[(long long)c * npts + f];
      }
      __syncthreads();
      if (tid == 0) P.tau[V] = tt;
      break;
    }
  } else if (tid == 0 && P.p_used) {
    P.p_used[tent] = (signed char)p;
  }

  // ---- 6. top values overwrite the stored values -----------------------------------
  for (int r = 0; r < m; ++r) {
    const double cr = gc[r], hr = gh[r];
    if constexpr (NS == 3) {
      if (Dp.ev_nl > 0 && (long long)(L.off_fg - L.off_W1) >= ev_doubles(p, Dp.ev_nl)) {
        // (v, sigma, U) at the top points on the matrix cores, 16 points per wave
        const int npts = (s_goff[r + 1] - s_goff[r]) * Q;
        const int nl = Dp.ev_nl, nat = Dp.ev_nat, nA16 = 16 * nat, ldb = ev_ldb(nl), P1 = p + 1;
        double* CMd = W1;
        double* PWW = W1 + (long long)(NS + 2) * nA16 * ldb;
        int* EXs = reinterpret_cast<int*>(PWW + 4 * 16 * 4 * P1);
        __syncthreads();
        for (int i = tid; i < nl; i += blockDim.x) EXs[i] = Dp.ev_ex[i];
        build_cm_dense<NS>(T, Dp, xs + r * NW, hr, CMd, nA16, ldb);
        double* pwv = PWW + wave * 16 * 4 * P1;
        // lane l < 16 holds the reference coordinates of its point of the next
        // block, loaded while the current block is evaluated
        double lamn[NS + 1];
        auto load_lam = [&](int blk) {
          const int f = min(blk + wave * 16 + lane, npts - 1);
#pragma unroll
          for (int k = 0; k <= NS; ++k) lamn[k] = gload(P.lam_ref + (size_t)(f % Q) * (NS + 1) + k);
        };
        if (lane < 16) load_lam(0);
        for (int blk = 0; blk < npts; blk += 64) {
          if (lane < 16) {
            const int f = min(blk + wave * 16 + lane, npts - 1);
            const double* R = EL + s_gel[s_goff[r] + f / Q] * ELS;
            const int lV = (int)R[El<NS>::LV];
            double var[NS + 1], phi = 0.0;
            for (int d = 1; d <= NS; ++d) var[d] = 0.0;
            for (int k = 0; k <= NS; ++k) {
              phi += lamn[k] * R[El<NS>::TAU + k];
              for (int d = 0; d < NS; ++d) var[1 + d] += lamn[k] * R[El<NS>::X + k * NS + d];
            }
            double lv = lamn[0];
#pragma unroll
            for (int k = 1; k <= NS; ++k)
              if (k == lV) lv = lamn[k];
            phi += lv * dt;
            var[0] = cr * (phi - tmid) / hr;
            for (int d = 0; d < NS; ++d) var[1 + d] = (var[1 + d] - XV[d]) / hr;
            for (int v = 0; v <= NS; ++v) {
              double a = 1.0;
              for (int e = 0; e < P1; ++e) {
                pwv[(lane * 4 + v) * P1 + e] = a;
                a *= var[v];
              }
            }
            if (blk + 64 < npts) load_lam(blk + 64);
          }
          wave_sync();
          double val[NS + 2][4];
          eval16_mfma<NS + 2, NS + 1>(CMd, nA16, ldb, nl, nat, Dp.ev_nks, Dp.ev_nkv, EXs, pwv, P1, val);
          if ((lane & 15) == 0) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
              const int f = blk + wave * 16 + (lane >> 4) + 4 * rr;
              if (f < npts) {
                const double* R = EL + s_gel[s_goff[r] + f / Q] * ELS;
                const int q = f % Q;
                const int e = (int)R[El<NS>::E];
                double* st = P.state + (size_t)e * (NS + 2) * Q;
                st[q] = cr * val[0][rr];
#pragma unroll
                for (int d = 0; d < NS; ++d) st[(1 + d) * Q + q] = val[1 + d][rr];
                st[(NS + 1) * Q + q] = a0[r] + val[NS + 1][rr];
                bool fin = true;
#pragma unroll
                for (int c = 0; c < NS + 2; ++c) fin = fin && isfinite(val[c][rr]);
                if (!fin) atomicOr(P.status, kStatNan);
              }
            }
          }
          wave_sync();
        }
        continue;
      }
    }
    __syncthreads();
    for (int row = tid; row < (NS + 2) * T.M; row += blockDim.x) {
      double acc = 0.0;
      for (int e = T.tr_ptr[row]; e < T.tr_ptr[row + 1]; ++e) acc += T.tr_coef[e] * xs[r * NW + T.tr_j[e]];
      cm[row] = row >= (NS + 1) * T.M ? acc * hr : acc;
    }
    __syncthreads();
    const int npts = (s_goff[r + 1] - s_goff[r]) * Q;
    for (int f = tid; f < npts; f += blockDim.x) {
      const int li = s_gel[s_goff[r] + f / Q];
      const int q = f % Q;
      const double* R = EL + li * ELS;
      const int lV = (int)R[El<NS>::LV];
      const double* lam = P.lam_ref + (size_t)q * (NS + 1);
      double xt[NS], phi = 0.0;
      for (int d = 0; d < NS; ++d) xt[d] = 0.0;
      for (int k = 0; k <= NS; ++k) {
        phi += lam[k] * R[El<NS>::TAU + k];
        for (int d = 0; d < NS; ++d) xt[d] += lam[k] * R[El<NS>::X + k * NS + d];
      }
      phi += lam[lV] * dt;
      double var[NS + 1];
      var[0] = cr * (phi - tmid) / hr;
      for (int d = 0; d < NS; ++d) var[1 + d] = (xt[d] - XV[d]) / hr;
      double val[NS + 2];
#pragma unroll
      for (int c = 0; c < NS + 2; ++c) val[c] = 0.0;
      eval_runs<NS, true>(T, runs, var, cm, val);
      const int e = (int)R[El<NS>::E];
      double* st = P.state + (size_t)e * (NS + 2) * Q;
      st[q] = cr * val[0];
#pragma unroll
      for (int d = 0; d < NS; ++d) st[(1 + d) * Q + q] = val[1 + d];
      st[(NS + 1) * Q + q] = a0[r] + val[NS + 1];
      bool fin = true;
#pragma unroll
      for (int c = 0; c < NS + 2; ++c) fin = fin && isfinite(val[c]);
      if (!fin) atomicOr(P.status, kStatNan);
    }
  }
  __syncthreads();
  if (tid == 0) P.tau[V] = tt;
  break;
  }  // degree attempts
}

// All tents of one layer: tents t0 .. t0+count-1.  Without a counter each
// workgroup solves tent t0 + blockIdx.x; with a counter (persistent mode) a
// resident grid takes tents in queue order from the counter until it passes
// count (every workgroup exits after at most count + gridDim.x draws).
template <int NS, int TPW, bool MIXED, bool MOM = false>
__global__ __launch_bounds__(kBlock) void tent_layer_kernel(KParams P, LdsPlan L, int t0, int count, int* ctr) {
  extern __shared__ double lds[];
  if (ctr == nullptr) {
    const int qi = t0 + blockIdx.x;
    solve_tent<NS, TPW, MIXED, MOM>(P, L, P.order ? P.order[qi] : qi, lds);
    return;
  }
  __shared__ int s_next;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(ctr, 1);
    __syncthreads();
    const int i = s_next;
    __syncthreads();
    if (i >= count) break;
    solve_tent<NS, TPW, MIXED, MOM>(P, L, P.order ? P.order[t0 + i] : t0 + i, lds);
    __syncthreads();
  }
}

namespace {

template <int NS, bool MX>
const void* kernel_ptr_mx(int tpw) {
  switch (tpw) {
    case 1:
      return (const void*)tent_layer_kernel<NS, 1, MX>;
    case 2:
      return (const void*)tent_layer_kernel<NS, 2, MX>;
    case 4:
      return (const void*)tent_layer_kernel<NS, 4, MX>;
    case 8:
      return (const void*)tent_layer_kernel<NS, 8, MX>;
    default:
      return (const void*)tent_layer_kernel<NS, 16, MX>;
  }
}

template <int NS>
// tpw = 0 selects the moment-mode kernel (FP64, no Gram tiles)
const void* kernel_ptr(int tpw, bool mixed) {
  if (tpw == 0) return (const void*)tent_layer_kernel<NS, 1, false, true>;
  return mixed ? kernel_ptr_mx<NS, true>(tpw) : kernel_ptr_mx<NS, false>(tpw);
}

template <int NS, bool MX>
hipError_t launch_mx(const KParams& P, const LdsPlan& L, int t0, int count, int grid_n, int* ctr, hipStream_t stream) {
  dim3 grid(grid_n), block(kBlock);
  size_t shm = (size_t)L.total * sizeof(double);
  if (L.moment && !MX) {
    hipLaunchKernelGGL((tent_layer_kernel<NS, 1, false, true>), grid, block, shm, stream, P, L, t0, count, ctr);
    return hipGetLastError();
  }
  switch (L.TPW) {
    case 1:
      hipLaunchKernelGGL((tent_layer_kernel<NS, 1, MX>), grid, block, shm, stream, P, L, t0, count, ctr);
      break;
    case 2:
      hipLaunchKernelGGL((tent_layer_kernel<NS, 2, MX>), grid, block, shm, stream, P, L, t0, count, ctr);
      break;
    case 4:
      hipLaunchKernelGGL((tent_layer_kernel<NS, 4, MX>), grid, block, shm, stream, P, L, t0, count, ctr);
      break;
    case 8:
      hipLaunchKernelGGL((tent_layer_kernel<NS, 8, MX>), grid, block, shm, stream, P, L, t0, count, ctr);
      break;
    default:
      hipLaunchKernelGGL((tent_layer_kernel<NS, 16, MX>), grid, block, shm, stream, P, L, t0, count, ctr);
      break;
  }
  return hipGetLastError();
}

template <int NS>
hipError_t launch_ns(const KParams& P, const LdsPlan& L, int t0, int count, int grid_n, int* ctr, hipStream_t stream) {
  return P.precision ? launch_mx<NS, true>(P, L, t0, count, grid_n, ctr, stream)
                     : launch_mx<NS, false>(P, L, t0, count, grid_n, ctr, stream);
}

template <int NS>
hipError_t smem_ns(size_t bytes) {
  const hipFuncAttribute a = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e = hipSuccess;
  for (int mx = 0; mx < 2 && e == hipSuccess; ++mx)
    for (int tpw : {1, 2, 4, 8, 16})
      if (e == hipSuccess) e = hipFuncSetAttribute(kernel_ptr<NS>(tpw, mx == 1), a, (int)bytes);
  if (e == hipSuccess) e = hipFuncSetAttribute(kernel_ptr<NS>(0, false), a, (int)bytes);
  return e;
}

}  // namespace

int launch_layer(const KParams& P, const LdsPlan& L, int t0, int count, int grid_n, int* ctr, void* stream_) {
  if (count <= 0) return 0;
  hipStream_t stream = (hipStream_t)stream_;
  if (!ctr) grid_n = count;
  hipError_t e;
  switch (P.n) {
    case 1:
      e = launch_ns<1>(P, L, t0, count, grid_n, ctr, stream);
      break;
    case 2:
      e = launch_ns<2>(P, L, t0, count, grid_n, ctr, stream);
      break;
    default:
      e = launch_ns<3>(P, L, t0, count, grid_n, ctr, stream);
      break;
  }
  return e == hipSuccess ? 0 : -1;
}

int resident_blocks_per_cu(int n, int tpw, bool mixed, size_t shm_bytes) {
  const void* k = n == 1 ? kernel_ptr<1>(tpw, mixed) : n == 2 ? kernel_ptr<2>(tpw, mixed) : kernel_ptr<3>(tpw, mixed);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kBlock, shm_bytes) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

int set_kernel_smem_limit(int n, size_t bytes) {
  hipError_t e;
  switch (n) {
    case 1:
      e = smem_ns<1>(bytes);
      break;
    case 2:
      e = smem_ns<2>(bytes);
      break;
    default:
      e = smem_ns<3>(bytes);
      break;
  }
  return e == hipSuccess ? 0 : -1;
}

}  // namespace tdg
