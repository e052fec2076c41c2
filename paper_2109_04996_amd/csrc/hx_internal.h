// Internal declarations shared by the hexpa sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "hexpa.h"

namespace hx {

constexpr int kMaxP = 9;   // nodes per direction (degree 8)
constexpr int kStrip = 8;  // longest strip (elements): the stride of the strip element lists
constexpr int kStripP = 8; // the Gauss-point mass kernel uses strips at this many nodes per direction
// Strip scatter (an element's P^2 node lines must fit one wavefront). The collocated kernel uses
// strips at P = 3, 4, 5 and 8 nodes per direction: at P = 6 and 7 (one element per wavefront
// with 28 and 15 lanes idle) the one-element-per-workgroup kernel measured faster. The Gauss-point
// kernel uses them for mass at P = 8 and for scalar diffusion with q = 8 at P = 7 and 8 (its 166
// registers allow one eight-wavefront workgroup per CU, against twelve one-wavefront ones without
// strips: p = 7 gains 9%, p = 6 1.5%, and three components lose 1.5%).
constexpr bool colloc_strips(int P) { return (P >= 3 && P <= 5) || P == 8; }
constexpr bool gauss_strips(int P, int Q, bool mass, int NC) {
  return mass ? (P == 8 && NC == 1) : (NC == 1 && Q == 8 && (P == 7 || P == 8));
}
constexpr bool strip_degree(int P) { return colloc_strips(P) || P == 7; }  // the mesh builds strips
constexpr int kMinStripsPerColor = 512;  // collocated strips below P = 8: at least this many strip groups (workgroups) per color on average
// elements per strip for P nodes per direction: seven for P = 3 (they fill one wavefront), else kStrip
constexpr int strip_len(int P) { return P == 3 ? 7 : kStrip; }
constexpr int kMaxQ = 10;  // quadrature points per direction

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
hx_status fail(hx_status code, const std::string &msg);
hx_status hip_fail(hipError_t e, const char *what);

#define HX_HIP(call)                                   \
  do {                                                 \
    hipError_t _e = (call);                            \
    if (_e != hipSuccess) return hx::hip_fail(_e, #call); \
  } while (0)

// ---------------------------------------------------------------- device buffers
template <typename T>
struct DevBuf {
  T *ptr = nullptr;
  size_t count = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    count = 0;
  }
  hipError_t alloc(size_t n) {
    release();
    count = n;
    if (n == 0) return hipSuccess;
    return hipMalloc(reinterpret_cast<void **>(&ptr), n * sizeof(T));
  }
  hipError_t upload(const T *h, size_t n) {
    hipError_t e = alloc(n);
    if (e != hipSuccess || n == 0) return e;
    return hipMemcpy(ptr, h, n * sizeof(T), hipMemcpyHostToDevice);
  }
};

// ---------------------------------------------------------------- 1D basis (host, FP64)
struct Basis1D {
  int p = 0, P = 0, q = 0, rule = HX_GAUSS;
  std::vector<double> nodes, qpts, qw;
  std::vector<double> interp;  // [q][P]
  std::vector<double> grad;    // [q][P]
  std::vector<double> colloc;  // [q][q]: derivative of the Lagrange basis on the q points, at those points
};

bool make_basis(int p, int q, int rule, Basis1D &out, std::string &err);
void gll_nodes_weights(int p, std::vector<double> &x, std::vector<double> &w);
void gauss_nodes_weights(int q, std::vector<double> &x, std::vector<double> &w);
void lagrange_tables(const std::vector<double> &nodes, const std::vector<double> &pts,
                     std::vector<double> &val, std::vector<double> &der);

}  // namespace hx

struct hx_basis_s {
  hx::Basis1D b;
};

struct hx_mesh_s {
  int p = 0, P = 0, device = 0;
  int64_t nelem = 0, nnodes = 0, nfree = 0, nuntouched = 0;
  int ncolors = 0;
  std::vector<int32_t> order;        // internal position -> caller element id
  std::vector<int64_t> color_start;  // ncolors + 1
  std::vector<double> h_xyz;         // nnodes*3
  hx::DevBuf<int32_t> idx;           // [E_internal][P^3] node ids
  hx::DevBuf<int32_t> idx_rows;      // [E_internal][P^2] first id of each r1-row (empty unless all rows are runs)
  hx::DevBuf<int32_t> idx_affine;    // [E_internal][4] {base, s_j, s_k, 0}: node (i,j,k) = base + i + j s_j + k s_k
                                     // (empty unless every element is numbered that way)
  hx::DevBuf<uint16_t> own;          // [E_internal][P^2] bit k: this element writes node (i,j,k) first
  hx::DevBuf<int32_t> order_d;       // internal position -> caller element id
  hx::DevBuf<double> xyz;            // nnodes*3
  hx::DevBuf<uint8_t> freemask;      // nnodes, 1 = free node
  hx::DevBuf<double> zeros;          // 64 zeros: target of masked read-modify-write loads
  // strips: chains of up to kStrip elements, each sharing its r1 = +1 face with the next one's
  // r1 = -1 face, scattered together by one workgroup of the collocated kernel. Strips have
  // their own coloring (no two strips of a color share a node) and ownership bits; element ids
  // are internal positions. Empty unless strip_degree(P) and the mesh has such chains.
  // Whole strips of one color are packed into groups of up to strip_len(P) elements, one workgroup each.
  int nstrip_colors = 0;
  int64_t nstrips = 0, nstrip_groups = 0;
  std::vector<int64_t> strip_color_start;  // nstrip_colors + 1, in groups
  hx::DevBuf<int32_t> strip_elems;         // [nstrip_groups][kStrip], -1 past the group's last element
  hx::DevBuf<uint8_t> strip_link;          // [nstrip_groups] bit w: slot w + 1 continues slot w's strip
  hx::DevBuf<uint16_t> strip_own;          // [E_internal][P^2] bit k: first write of node (i,j,k) in strip order
  // transpose of the element restriction (made on first use): the E-vector slots e*P^3 + l (caller
  // element e, local node l) of each node, ascending; gather_ptr has nnodes + 1 entries
  hx::DevBuf<int32_t> gather_ptr, gather_slot;
  // the same in internal element order: slots e * P^3 + l (internal position e), ascending (made on first use)
  hx::DevBuf<int32_t> slot_ptr, slot_idx;
  int index_mode = 0;  // 0 full index array, 1 one id per r1-row, 2 affine numbering
  // A host-only plan (hx_mesh_plan) holds no device memory: the arrays the device buffers would hold stay
  // on the host for inspection, and operators reject the mesh.
  bool host_only = false;
  std::vector<int32_t> h_idx, h_strip_elems;
  std::vector<uint16_t> h_own, h_strip_own;
  std::vector<uint8_t> h_strip_link;
};

struct hx_op_s {
  hx_op_s() = default;
  hx_op_s(const hx_op_s &) = delete;
  hx_op_s &operator=(const hx_op_s &) = delete;
  ~hx_op_s() {
    if (solve_stream) (void)hipStreamDestroy(solve_stream);
  }
  hipStream_t solve_stream = nullptr;  // the solver's own stream (graph capture), made on first use
  hx_mesh mesh = nullptr;
  hx::Basis1D b;
  int kind = 0, ncomp = 1, P = 0, Q = 0;
  bool colloc = false;  // diffusion on the GLL nodes: no interpolation step
  int ncq = 1;          // stored values per quadrature point
  hx::DevBuf<double> qdata;    // [E_internal][ncq][Q^3]
  hx::DevBuf<float> qdata32;   // FP32 copy, made on demand
  // HX_HELMHOLTZ: qdata holds alpha times the diffusion factors; qmass [E_internal][Q^3] beta w detJ
  double alpha = 1.0, beta = 0.0;
  hx::DevBuf<double> qmass;
  hx::DevBuf<float> qmass32;   // FP32 copy, made with qdata32
  hx::DevBuf<double> tab;      // device 1D tables: interp [Q][P], grad [Q][P], colloc [Q][Q]
  hx::DevBuf<float> tab32;
  // solver workspace (allocated on first solve)
  hx::DevBuf<double> work;
  hx::DevBuf<float> work32;
  hx::DevBuf<double> red;      // reduction partials and device scalars
  hx::DevBuf<double> diag;     // assembled diagonal (cached)
  hx::DevBuf<double> evec;     // E-vector of the node-gather apply inside solves (made on first use)
  bool diag_valid = false;
  // coefficient parameters (kept for the element features of the learned preconditioner)
  int kappa_M = 0;
  std::vector<double> kappa_omega, kappa_phase;
  double kappa_scale = 0.0, kappa_shift = 0.0;
  // learned preconditioner: element features and work buffers (made on first use)
  bool mlp_ready = false;
  hx::DevBuf<float> mlp_logk;      // [n] log kappa at the nodes
  hx::DevBuf<uint16_t> mlp_feat16; // [E_internal][P^3] centred log kappa (marker on constrained nodes), bf16
  hx::DevBuf<float> mlp_dis;       // [n] D^-1/2 on free nodes, 0 on constrained ones
  hx::DevBuf<float> mlp_wmult;     // [n] 1 / multiplicity on free nodes, 0 on constrained ones
  hx::DevBuf<uint16_t> mlp_x16, mlp_h16;
  bool mlp_x16_feat = false;       // the coefficient half of the mlp_x16 rows is written
  hx::DevBuf<float> mlp_dw;        // [n] D^-1/2 w (the output gather's node factor)
  hx::DevBuf<double> mlp_dinv;     // [n] D^-1 on free nodes, 0 on constrained ones
  hx::DevBuf<float> mlp_y, mlp_rnorm;
  // HX_LOR: the assembled low-order refined matrix, ELL [lor_w][nnodes] (column-major)
  int lor_w = 0;
  hx::DevBuf<int32_t> lor_col;
  hx::DevBuf<double> lor_val;
  // bf16 matrix-core operator: FP32 tables and a bfloat16 copy of qdata (made on demand)
  hx::DevBuf<float> tab_bf16;
  hx::DevBuf<uint16_t> qdata_bf16;
};

// p-multigrid hierarchy: level 0 finest. Level l (l < L-1) also holds the transfer to level l+1.
struct hx_pmg_s {
  struct Level {
    hx_op op = nullptr;
    int64_t n = 0;
    double lam_max = 0.0;
    int64_t applies = 0;      // operator applies made by V-cycles on this level
    hx::DevBuf<double> work;  // 10 n: the level's vectors
    hx::DevBuf<float> work32; // 10 n: the level's FP32 vectors (FP32 V-cycle)
    hx::DevBuf<double> red;   // reduction partials and device scalars of its solves
    // transfer from level l+1 (coarse) to this level (fine); empty on the coarsest level
    int Pc = 0;
    hx::DevBuf<double> interp;     // [Pf][Pc]: coarse Lagrange basis at the fine GLL nodes
    hx::DevBuf<int32_t> cmap;      // [E] fine internal position -> coarse internal position
    hx::DevBuf<double> ecoarse;    // [E][Pc^3] coarse E-vector of a restriction (coarse internal order; FP32 ones
                                   // use the front half)
    hx::DevBuf<int64_t> csr_ptr;   // [n_coarse + 1]
    hx::DevBuf<int32_t> csr_slot;  // E-vector slots of each coarse node, ascending
  };
  hx_pmg_s() = default;
  hx_pmg_s(const hx_pmg_s &) = delete;
  hx_pmg_s &operator=(const hx_pmg_s &) = delete;
  ~hx_pmg_s() {
    if (hS) (void)hipHostFree(hS);
  }
  hx_pmg_opts opts{};
  std::vector<std::unique_ptr<Level>> lv;
  double *hS = nullptr;  // pinned host scalars of the coarse solve
};

namespace hx {

// ---------------------------------------------------------------- kernels (launchers)
struct ApplyArgs {
  const int32_t *idx;
  const uint16_t *own;
  const void *qd;       // double or float
  const double *tab;    // device tables (double)
  const float *tab32;
  const void *x;
  void *y;
  const int32_t *order;  // for E-vector output
  int64_t e_begin, e_end;
  int64_t nnodes;
};

enum class Prec { F64, F32_Q64, F32_Q32 };

// one launch per color; out_elem: write the E-vector instead of scattering
hx_status launch_apply(const hx_op_s &op, Prec prec, bool out_elem, const ApplyArgs &a, hipStream_t s);
hx_status launch_setup_qdata(hx_op_s &op, const hx_kappa_rff *kappa, hipStream_t s, int *bad_det);
hx_status launch_diagonal(hx_op_s &op, double *diag, hipStream_t s);
hx_status launch_diagonal_tables(const hx_op_s &op, const double *interp, const double *grad, double *diag,
                                 hipStream_t s);
hx_status launch_apply_bf16(hx_op_s &op, bool split, const float *x, float *y, hipStream_t s);
// the low-order refined operator: y = L x (FP64 L-vectors) and its diagonal
hx_status lor_apply(const hx_op_s &op, const double *x, double *y, hipStream_t s);
hx_status lor_diagonal(const hx_op_s &op, double *diag, hipStream_t s);
// the mesh's transpose restriction (gather_ptr, gather_slot), built on first call
hx_status mesh_gather_csr(hx_mesh_s &m);
// the node -> element slot table in internal element order (slot_ptr, slot_idx), built on first call
hx_status mesh_slots(hx_mesh_s &m);
// p-multigrid transfer between level l (fine) and l+1 on FP64 or FP32 vectors; fm: free mask applied to the
// output, or null
template <typename T>
hx_status launch_prolong(const hx_pmg_s &mg, int l, const T *xc, T *yf, const uint8_t *fm, hipStream_t s);
// rb: when given, the restriction acts on the fine residual m (rb - rf) (m the fine free mask)
template <typename T>
hx_status launch_restrict(const hx_pmg_s &mg, int l, const T *rf, T *yc, const uint8_t *fm, hipStream_t s,
                          const T *rb = nullptr);
// each level's diagonal and lam_max (solver side)
hx_status pmg_setup_levels(hx_pmg_s &mg, hipStream_t s);

}  // namespace hx
