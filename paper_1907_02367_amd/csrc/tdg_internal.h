// Internal data structures shared by the libtdg host code and its HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "tdg.h"

namespace tdg {

constexpr int kMaxP = 10;        // highest degree of U^p with tables
// moment task (a run of up to 4 monomials that differ only in the exponent of the
// last variable, consecutive): word 0 = prefix exponents e0 | e1 << 5 | e2 << 10
// (variables 0..n-1) | first last-variable exponent << 15; words 1, 2 = the run's
// monomial indices, 16 bits each (0xFFFF past the run)
constexpr int kTaskInts = 3;
constexpr int kTaskSlots = 6;   // moment-monomial tasks per thread held in registers (<= kTaskSlots * kBlock)
constexpr int kTaskSlots1 = 2;  // tasks over the monomials of degree <= p, per thread
// Top moments on the FP64 matrix cores (3+1D moment Gram): the moment monomial
// t^k x1^a1 x2^a2 x3^a3 is L(t, x1) R(x2, x3); over the points of one element
// the moments of all products form the 16x16 tiles of (w L)^T R, only the tiles
// with a product of degree <= 2p-2 are formed, at most kMomTileSlots per wave
constexpr int kMomTileSlots = 6;
constexpr int kMaxGroups = 32;   // speed groups inside one tent (Sec. 4.2)
constexpr int kMaxPatch = 64;    // elements in one vertex patch
constexpr int kMaxFaces = 64;    // Dirichlet facets containing one vertex
constexpr int kBlock = 256;      // threads per workgroup of the tent kernels
// degree network: features, hidden width, outputs (log indicator for p = 2..8)
constexpr int kFeat = 8;
constexpr int kHid = 64;
constexpr int kOut = 7;
constexpr int kNParam = kHid * kFeat + kHid + kHid * kHid + kHid + kOut * kHid + kOut;
// samples one call of the allocation-free network gradient can take (its fixed
// device scratch holds the partial gradients of kNoAllocMaxSamples / 32 blocks)
constexpr long long kNoAllocMaxSamples = 8192;

// Sparse tables of the Trefftz basis of U^p (c = 1) over the monomials
// t^k x^alpha, k + |alpha| <= p, ordered by total degree, so the first M1
// monomials are those of degree <= p - 1.  Monomial i > 0 is
// mono[parent[i]] * (t if var[i] == 0 else x_var[i]).
// First-order table (v, sigma) = (dU/dt, -grad U): CSR over rows j*(n+1)+comp
// for the non-constant functions j = 0..NW-1 (basis functions 1..N-1).
// U table: CSR over rows j (basis function j+1).
struct TableDesc {
  int p, NW, M, M1, M2, fo_nnz, u_nnz, ue_n, tr_n;
  int pch, nwp, pci;  // execution plan at this degree: points per chunk, operand stride, face chunk
  int mpch, moff;     // 3+1D moment phase: points per chunk and (>= 0) its regions' offset in W1
  const int* expo2;  // M2*(n+1) exponents of the moment monomials (degree <= 2p-2)
  const int* K2;     // M1*M1: moment index of the product of monomials k, l < M1
  const int* task2;  // ntask2 moment tasks over the moment monomials (degree <= 2p-2)
  const int* task1;  // ntask1 moment tasks over the monomials of degree <= p
  int ntask2, ntask1;
  // matrix-core top moments (3+1D): mt_ntile tiles (0: not used at this degree);
  // per tile and lane l%16 the packed exponents a0 | a1 << 5 (row 16 I + l%16 of
  // the L list) | c0 << 10 | c1 << 15 (column 16 J + l%16 of the R list):
  // mt_ex[tile*16 + l%16]; mt_map[tile*256 + row*16 + col] = moment index or -1
  int mt_ntile;
  const int* mt_ex;
  const int* mt_map;
  // matrix-core evaluation of the solution at points (3+1D): monomial k of
  // degree <= p is L_a(t, x1) R_b(x2, x3); ev_ab[k] = a | b << 16; ev_ex[i] =
  // e_first | e_second << 8 of entry i of the (shared) two-variable list of
  // degree <= p (ev_nl entries, by degree); ev_nat tiles of 16 L entries, tile I
  // needs ev_nks[I] steps of 4 R entries; ev_nl = 0: not used at this degree
  // (ev_nkv[I]: the same for v and sigma, whose degree is at most p - 1)
  int ev_nl, ev_nat, ev_nks[8], ev_nkv[8];
  const int* ev_ab;
  const int* ev_ex;
  // entry form: entries of basis function j+1 are ue_ptr[j]..ue_ptr[j+1]-1; entry e
  // holds (n+2) pairs (monomial index, coefficient) for U, v = dU/dt and
  // sigma_m = -dU/dx_m: ue_idx[e*(n+2)+s], ue_coef[e*(n+2)+s] (coefficient 0 if absent)
  const int* ue_ptr;
  const int* ue_idx;
  const double* ue_coef;
  // transposed form for the write-back: row comp*M + mono (comp 0 = v, 1..n = sigma,
  // n+1 = U) lists (function j, coefficient): tr_ptr, tr_j, tr_coef
  const int* tr_ptr;
  const int* tr_j;
  const double* tr_coef;
  const int* parent;
  const int* var;
  const int* expo;  // M*(n+1) exponents (k, alpha) of each monomial
  const int* fo_ptr;
  const int* fo_idx;
  const double* fo_coef;
  const float* fo_coef32;
  const int* u_ptr;
  const int* u_idx;
  const double* u_coef;
};

// Everything a tent kernel reads or writes.  All pointers are device pointers.
struct KParams {
  int n, nv, ne, Q, pmax, ntents;
  int precision;     // 0 fp64, 1 mixed
  int recover_U;
  double alpha, beta;
  // static geometry
  const double* coords;    // nv*n
  const double* c;         // ne
  const double* grad_lam;  // ne*(n+1)*n
  const double* absdet;    // ne
  const double* lam_ref;   // Q*(n+1)
  const double* w_ref;     // Q
  const int* elems;        // ne*(n+1)
  const int* v2e_ptr;      // nv+1
  const int* v2e;
  const int* vb_ptr;       // nv+1: Dirichlet boundary facets containing V
  const int* vb;           // pairs (element, local index of the opposite vertex)
  const int* vn_ptr;       // nv+1: Neumann boundary facets containing V
  const int* vn;           // pairs, as vb
  const int* vi_ptr;       // nv+1: speed-interface facets containing V
  const int* vi;           // quadruples (e1, k1, e2, k2), e1 < e2
  // tents
  const int* tent_V;
  const double* tent_tb;
  const double* tent_tt;
  const long long* bpt_off;  // ntents+1 offsets into gD
  const signed char* p_per_tent;  // nullable
  // nullable: the order in which a layer's tents are drawn (queue position
  // t0 + i -> tent order[t0 + i]; a permutation of the layer), costliest first
  const int* order;
  int p_fixed;                    // > 0 and no p_per_tent: every tent at this degree
  // dynamic state
  double* state;  // ne * (n+2) * Q, element-major, then component, then point
  double* tau;    // nv
  const double* gD;
  int* status;    // device error word
  double* dissip; // ntents, nullable
  int* ir_steps;  // ntents, nullable (mixed precision)
  int indicator;      // 1: compute the per-tent indicator into dissip
  int write_back;     // 0: indicator only (state and front untouched)
  double eta_tol;     // > 0: re-solve at p_max where the indicator exceeds it
  signed char* p_used;  // nullable: degree each tent was finally solved with
  double* work;   // global scratch for systems that do not fit in LDS
  long long work_stride;  // doubles per workgroup slot
  const TableDesc* tabd;  // device array indexed by the degree (0 .. kMaxP)
};

// Device status bits (OR-ed by kernels)
enum : int {
  kStatSingular = 1,
  kStatNan = 2,
  kStatPatch = 4,
  kStatGroups = 8,
  kStatNoConv = 16,
  kStatSize = 32,
};

// LDS layout of the tent kernel (sizes in doubles), chosen on the host.
struct LdsPlan {
  int S;         // largest system size (groups * NW)
  int lda;       // row stride of the augmented matrix
  int NWP;       // row stride of the Gram operand (16-padded NW, odd)
  int PCH;       // points per chunk at p_max
  int pch[kMaxP + 1];  // points per chunk at each degree (>= PCH below p_max)
  int nwp[kMaxP + 1];  // Gram operand row stride at each degree
  int M;         // monomials of degree <= p_max
  int TPW;       // Gram tiles per wave
  int maxpatch;
  int ELS;       // doubles per patch element record
  int A_in_lds;  // 1: system in LDS; 0: in the global scratch slot of the workgroup
  int tab_in_lds;
  int tab_int_dbl;  // doubles occupied by the integer part of a staged table
  int maxfaces;  // Dirichlet facets containing one vertex, at most
  int moment;    // 1: Gram and right-hand sides from point moments of the monomials
  int pci[kMaxP + 1];  // points per chunk of the interface faces at each degree
  int lu_nb;     // panel width of the blocked LU of a system in global memory (0: unblocked)
  // 3+1D moment phase at degree p: a larger chunk (mpch points) whose point and
  // power regions sit in the part of W1 the degree's moments leave free (moff,
  // doubles from W1), or moff = -1: the chunk regions of p_max
  int mpch[kMaxP + 1], moff[kMaxP + 1];
  int off_A, off_x, off_tab, off_el, off_misc, off_pt, off_pow, off_mono, off_W1, off_fg, off_AF, off_vec, total;
};

// LDS doubles of the matrix-core evaluation at degree p (3+1D): the dense
// coefficients of the n+2 fields over (L entry, R entry) pairs, the powers of
// 16 points per wave (4 waves, n+1 variables, exponents 0..p), the entry list
constexpr int ev_ldb(int nl) { return nl | 1; }
// k-steps of 4 entries held in registers by the evaluation: ceil(66 / 4) covers
// the two-variable list of degree 10
constexpr int kEvalMaxSteps = 17;
constexpr long long ev_doubles(int p, int nl) {
  return 5LL * (16 * ((nl + 15) / 16)) * ev_ldb(nl) + 4LL * 16 * 4 * (p + 1) + (nl + 1) / 2 + 1;
}

// LDS workspace (doubles) of the blocked LU of an S x (S+1) system with panels
// of nb columns: the panel (column stride S|1), the U12 rows (row stride
// (S+1)|1), then S + nb + 1 ints (row origins, pivots, one spare).
constexpr int lu_ldp(int S) { return S | 1; }
constexpr int lu_ldu(int S) { return (S + 1) | 1; }
constexpr long long lu_ws_doubles(int S, int nb) {
  return (long long)nb * (lu_ldp(S) + lu_ldu(S)) + (S + nb + 2) / 2;
}

int launch_layer(const KParams& P, const LdsPlan& L, int t0, int count, int grid_n, int* ctr, void* stream);
int resident_blocks_per_cu(int n, int tpw, bool mixed, size_t shm_bytes);  // tpw 0: moment-mode kernel
int set_kernel_smem_limit(int n, size_t bytes);
int launch_fill(double* p, double v, long long n, void* stream);
int launch_fill_i8(signed char* p, signed char v, long long n, void* stream);
int launch_features(const KParams& P, int t0, int count, float* feats, void* stream);
int launch_order(const signed char* p_sel, int t0, int count, int pmax, int* order, void* stream);
int launch_select(const unsigned short* wb, const float* feats, int t0, int count, float log_tol, int pmax,
                  signed char* p_sel, void* stream);
int launch_norms(const KParams& P, int kind, const double* ex, double* partial, int nblocks, double* out, void* stream);
int noalloc_scratch(float** out);  // device address of the fixed network-gradient scratch (current device)

// ---- host-side components ----------------------------------------------------
struct Topology {
  int n = 0, nv = 0, ne = 0;
  std::vector<double> coords;     // nv*n
  std::vector<int> elems;         // ne*(n+1)
  std::vector<double> c;          // ne
  std::vector<double> grad_lam;   // ne*(n+1)*n
  std::vector<double> absdet;     // ne
  std::vector<int> v2e_ptr, v2e;  // patches (ascending element)
  std::vector<int> nb_ptr, nb;    // neighbours (ascending)
  std::vector<int> vb_ptr, vb;    // Dirichlet boundary facets at V: (element, opposite local vertex)
  std::vector<int> vn_ptr, vn;    // Neumann boundary facets at V
  std::vector<std::pair<int, int>> bfacets;  // every boundary facet, ascending (element, local vertex)
  std::vector<int> vi_ptr, vi;    // interface facets at V
};

// Builds the topology; returns TDG_OK or an error code with a message.
int build_topology(const tdg_mesh& m, const double* c, Topology& T, std::string& err);

struct Quadrature {
  int n = 0, q = 0, Q = 0;
  std::vector<double> lam;  // Q*(n+1) barycentric coordinates
  std::vector<double> w;    // Q weights (sum 1/n!)
};
void gauss_jacobi01(int q, int a, std::vector<double>& x, std::vector<double>& w);
Quadrature simplex_rule(int n, int q);

struct Table {
  int n = 0, p = 0, NW = 0, M = 0, M1 = 0, M2 = 0;
  std::vector<int> expo2;  // M2*(n+1): exponents of the monomials of degree <= 2p-2
  std::vector<int> K2;     // M1*M1: index in expo2 of the product of monomials k and l
  std::vector<int> task2, task1;  // moment tasks (kTaskInts ints each) over expo2 and over expo
  int ntask2 = 0, ntask1 = 0;
  int mt_ntile = 0;                // matrix-core top-moment tiles (see TableDesc)
  std::vector<int> mt_ex, mt_map;
  int ev_nl = 0, ev_nat = 0, ev_nks[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // matrix-core evaluation (see TableDesc)
  int ev_nkv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<int> ev_ab, ev_ex;
  std::vector<int> parent, var;
  std::vector<int> expo;  // M*(n+1): k, alpha_1..alpha_n
  std::vector<int> fo_ptr, fo_idx;
  std::vector<double> fo_coef;
  std::vector<int> u_ptr, u_idx;
  std::vector<double> u_coef;
  std::vector<int> ue_ptr, ue_idx;
  std::vector<double> ue_coef;
  std::vector<int> tr_ptr, tr_j;
  std::vector<double> tr_coef;
};
Table build_table(int n, int p);

struct TentList {
  int n = 0;
  double T = 0, gamma = 0, max_slope = 0;
  std::vector<int> V;
  std::vector<double> tb, tt;
  std::vector<int64_t> layer_ptr;
};
int pitch_tents(const Topology& topo, double T, double gamma, TentList& out, std::string& err);

void set_error(const std::string& msg);

}  // namespace tdg

struct tdg_tents {
  tdg::TentList list;
};
