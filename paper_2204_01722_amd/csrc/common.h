// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/hpmg.h"

namespace hpmg {

// ---------------------------------------------------------------------------------
// Quadrature tiling.  Quadrature-point arrays (geometric factors, stored
// linearisation) are laid out [tile][field][ET * Q^3]: the ET consecutive elements of
// a tile are processed by one workgroup with one thread per quadrature point, so each
// field is read by one contiguous, fully coalesced sweep of the workgroup.
// ---------------------------------------------------------------------------------
constexpr int elems_per_tile(int Q) {
  return Q == 2 ? 32 : Q == 3 ? 9 : Q == 4 ? 4 : Q == 5 ? 2 : 1;
}
constexpr int tile_threads(int Q) {
  return ((elems_per_tile(Q) * Q * Q * Q + 63) / 64) * 64;
}

constexpr int NGEO = 10;    // W, dxi_k/dX_J (row-major)
// Stored linearisation per point: sqrt(W) dxi_k/dx_j (9), tau (xx yy zz yz xz xy),
// lambda log J.  Every use is W times a form bilinear in dxi/dx, so the weight rides in
// the scaled dxi/dx and is not stored (16 scalars instead of 17).
constexpr int NSTATE = 16;
constexpr int NINIT = 26;   // grad_X u (9), C^-1 (6), lambda log J (1), dxi/dx (9), J - 1 (1)

// Reference tables, in the operator's precision, at fixed offsets (max 8 x 8 each).
constexpr int TAB_B = 0;      // [Q][P] interpolation
constexpr int TAB_G = 64;     // [Q][P] reference derivative
constexpr int TAB_D = 128;    // [Q][Q] collocated derivative
constexpr int TAB_W = 192;    // [Q]    1D Gauss weights
constexpr int TAB_BB = 200;   // [Q][P] B*B   (elementwise, diagonal assembly)
constexpr int TAB_BG = 264;   // [Q][P] B*G
constexpr int TAB_GG = 328;   // [Q][P] G*G
constexpr int TAB_CTOF = 392; // [Pf][P] interpolation from this order to order Pf - 1,
                              // slot (Pf - 2) of 64 values, Pf = P+1 .. 6
constexpr int TAB_SIZE = 392 + 5 * 64;
__host__ __device__ constexpr int tab_ctof(int Pf) { return TAB_CTOF + (Pf - 2) * 64; }

// Element-to-node map used by the kernels: node id in the low 28 bits, the Dirichlet
// flags of the node's three components in bits 28..30.
constexpr uint32_t EMAP_ID_MASK = (1u << 28) - 1u;
constexpr int EMAP_BC_SHIFT = 28;
// Set on exactly one record of every node (its first record in element order): the
// element that writes the node in the p-transfers.
constexpr uint32_t EMAP_OWNER = 1u << 31;
constexpr int64_t MAX_NODES = int64_t(1) << 28;

constexpr int RED_BLOCKS = 512;  // fixed grid of the deterministic reductions

// Device scalar slots of a multigrid handle used by the fused Jacobi-PCG: r.z (2), r.r
// (3), breakdown flag (5), r.z of the current iteration, alternating (8, 9), stop flag
// (10), completed iterations (11), r.r of the start (12); per-iteration alpha and beta
// when recorded for the eigenvalue estimate (SC_ALPHA + k, SC_BETA + k, k < PCG_RECORD).
constexpr int SC_STOP = 10, SC_COUNT = 11, SC_RR0 = 12;
// Flexible CG (FP64, device scalars): p.q, r.r of the new residual, breakdown flag,
// alpha, z.r_new and z.r_old of the Polak-Ribiere beta, r.z alternating (FCG_RZ + 0, 1).
constexpr int FCG_PQ = 13, FCG_RR = 14, FCG_BRK = 15, FCG_ALPHA = 16, FCG_ZRN = 17, FCG_ZR = 18, FCG_RZ = 19;
constexpr int PCG_RECORD = 64;
constexpr int SC_ALPHA = 32, SC_BETA = SC_ALPHA + PCG_RECORD, SC_N = SC_BETA + PCG_RECORD;

}  // namespace hpmg

struct hpmg_op_s {
  int P = 0, Q = 0;
  int64_t E = 0, N = 0;
  const int32_t *elem_nodes = nullptr;
  const uint8_t *mask = nullptr;
  hpmg_op_s *fine = nullptr;  // non-null for coarse operators
  double mu = 0.0, lam = 0.0;
  const double *mu_e = nullptr, *lam_e = nullptr;
  int ET = 0, NQ = 0, NT = 0;
  int64_t tiles = 0;
  // workspace carve-up
  char *ws = nullptr;
  size_t ws_bytes = 0;
  double *tab64 = nullptr;
  float *tab32 = nullptr;
  uint32_t *emap = nullptr;
  double *geo = nullptr;       // fine only
  double *state64 = nullptr;   // fine only
  double *sinit = nullptr;     // fine only, caller-provided: [tile][26][ET*Q^3] (hpmg_state_initial)
  bool sinit_ready = false;
  float *state32 = nullptr;    // fine only
  double *scratch = nullptr;   // reductions
  int32_t *csr_off = nullptr;  // node -> incidences (element-local records), [N + 1]
  int32_t *csr_inc = nullptr;  // record index e * P^3 + a, sorted per node, [E * P^3]
  double *evec = nullptr;      // element output records [E][P^3][3] (FP64 or FP32)
  double *elmat = nullptr;     // P = 2 only: element matrices [E][300], upper triangle row-major (FP64 or FP32)
  int elmat_prec = -1;         // precision of the built element matrices (-1: none)
  uint64_t elmat_version = 0;  // state version they were built from
  uint64_t state_version = 0;  // fine operators: bumped at every stored linearisation
  unsigned *flags = nullptr;
  bool geo_ready = false, state_ready = false, state32_ready = false;
  void *host_extra = nullptr;  // host-side tables and scalars owned by the handle
};

namespace hpmg {

// Error reporting (thread-local message).
int fail(int status, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
#define HPMG_HIP(call)                                     \
  do {                                                     \
    hipError_t _e = (call);                                \
    if (_e != hipSuccess) return ::hpmg::hip_fail(_e, #call); \
  } while (0)

// Host tabulation (basis.cpp).
int tabulate(int P, int Q, double *B, double *G, double *D, double *xq, double *wq, double *gll);
int ctof_table(int Pf, int Pc, double *M);

// Launchers (op_kernels.hip / vec_kernels.hip).  All return hipError_t of the launch.
bool supported_pq(int P, int Q);
hipError_t launch_build_emap(const hpmg_op_s &op, hipStream_t s);
hipError_t launch_mark_owners(const hpmg_op_s &op, hipStream_t s);
// Stored-mode apply whose assembly also writes per-workgroup partials of du . y
// (ceil(N / 256) of them, in pq).  With `stop` set, every kernel of the apply returns at once while *stop != 0.
hipError_t launch_jacobian_dot(const hpmg_op_s &op, int prec, const void *du, void *y, double *pq,
                               const double *stop, hipStream_t s);
// Fused Jacobi-PCG iteration on the slots above; all kernels return at once while
// sc[SC_STOP] != 0.  update2 records alpha in *alpha_rec, dir2 beta in *beta_rec (when
// not null), counts the iteration in sc[SC_COUNT] and sets the stop flag on breakdown
// or when r.r <= rtol2 * sc[SC_RR0] (rtol2 < 0: never).
hipError_t launch_pcg_begin(double *sc, hipStream_t s);
// FCG steps on the slots above (FP64): update: alpha = r.z / p.q from the device
// scalars (0 on a breakdown, p.q <= 0 or r.z not finite, which sets sc[FCG_BRK]),
// x += alpha p, rn = r - alpha q, sc[FCG_RR] = rn.rn.  dir: beta = (z.rn - z.r) / r.z,
// r.z <- z.rn, p = z + beta p.  r.z of iteration `it` is read from FCG_RZ + (it & 1).
hipError_t launch_fcg_update(int64_t n, double *sc, int it, const double *p, const double *q, double *x,
                             const double *r, double *rn, double *partial, hipStream_t s);
hipError_t launch_fcg_dir(int64_t n, double *sc, int it, const double *z, double *p, hipStream_t s);
// The iteration on an order-1 operator assembled into 3 x 3 blocks (sliced ELL, width W,
// nn nodes): one launch replaces the element kernel, the fused assembly and dir2;
// ell_pcg_blocks(nn, node_major) workgroups write pq_part.  nn = 0 runs only the
// stopping test of the iteration before `it` (to close a batch).  node_major: blocks
// held entry-major over the nodes and a thread per node (else a node's rows contiguous
// and a thread per row), the same choice as the block build's (launch_ell_build).
// By default coarse levels of at least this many nodes are node-major.
constexpr int64_t ELL_NODE_MAJOR_MIN = 65536;
int ell_pcg_blocks(int64_t nn, bool node_major);
hipError_t launch_ell_pcg_apply(int prec, bool node_major, int64_t nn, int W, const int32_t *cols,
                                const void *vals, const void *z, const void *p_old, void *p_new, void *y, double *sc,
                                const double *partial, int it, double rtol2, double *pq_part, hipStream_t s);
// Assembles the order-1 element matrices of `op` (built in precision prec) into the
// sliced-ELL blocks; constrained rows become identity rows, constrained columns zero.
hipError_t launch_ell_build(const hpmg_op_s &op, int prec, bool node_major, int64_t W, const int32_t *cols,
                            void *vals, hipStream_t s);
hipError_t launch_pcg_update2(int prec, int64_t n, double *sc, int parity, int nb_pq, const double *pq_partial,
                              const void *p, const void *q, void *x, void *r, const void *dinv, void *z,
                              double *partial, double *alpha_rec, hipStream_t s);
hipError_t launch_pcg_dir2(int prec, int64_t n, double *sc, int parity, const double *partial, const void *z,
                           void *p, double rtol2, double *beta_rec, hipStream_t s);
hipError_t launch_inject(int64_t nc, const int32_t *map, const double *uf, double *uc, hipStream_t s);
hipError_t launch_state_initial(const hpmg_op_s &op, const double *u, hipStream_t s);
hipError_t launch_body_load(const hpmg_op_s &op, const double *g, double *f_ext, hipStream_t s);
hipError_t launch_traction_load(const hpmg_op_s &op, const double *X, int64_t nf, const int32_t *face_elem,
                                const int32_t *face_id, const double *t, double *rec, int32_t *rec_node,
                                hipStream_t s);
hipError_t launch_assemble_csr(int64_t N, const int32_t *off, const int32_t *inc, const double *rec,
                               const uint8_t *mask, double *y, hipStream_t s);
hipError_t launch_qdata(const hpmg_op_s &op, const double *coords, hipStream_t s);
hipError_t launch_residual(const hpmg_op_s &op, const double *u, double *r, bool store, hipStream_t s);
hipError_t launch_jacobian(const hpmg_op_s &op, int prec, int mode, const double *u, const void *du,
                           void *y, hipStream_t s);
hipError_t launch_diagonal(const hpmg_op_s &op, int prec, void *diag, hipStream_t s);
hipError_t launch_prolong_add(const hpmg_op_s &coarse, const hpmg_op_s &fine, int prec,
                              const void *xc, void *yf, hipStream_t s);
hipError_t launch_restrict(const hpmg_op_s &fine, const hpmg_op_s &coarse, int prec, const void *rf,
                           void *rc, hipStream_t s);
hipError_t launch_energy(const hpmg_op_s &op, const double *u, double *psi, hipStream_t s);
hipError_t launch_vjp(const hpmg_op_s &op, int prec, int mode, const double *u, const void *w, void *ub,
                      double *mub, double *lamb, hipStream_t s);
hipError_t launch_export_qdata(const hpmg_op_s &op, double *out, hipStream_t s);
hipError_t launch_elmat_build(const hpmg_op_s &op, int prec, hipStream_t s);

// Vector kernels.
hipError_t launch_init_bc(int prec, int64_t n_nodes, const uint8_t *mask, const void *x, void *y,
                          hipStream_t s);  // y = mask ? x : 0
hipError_t launch_cast_state(int64_t n, const double *a, float *b, hipStream_t s);
hipError_t launch_dot(int prec, int64_t n, const void *x, const void *y, double *partial,
                      double *out, hipStream_t s);
hipError_t launch_dot2(int prec, int64_t n, const void *x, const void *y, const void *z,
                       double *partial, double *out, hipStream_t s);  // out[0]=x.y, out[1]=z.z
hipError_t launch_sum(int64_t n, const double *x, double *partial, double *out, hipStream_t s);
hipError_t launch_axpby(int prec, int64_t n, double a, const void *x, double b, void *y, hipStream_t s);
hipError_t launch_waxpby(int prec, int64_t n, double a, const void *x, double b, const void *y,
                         void *w, hipStream_t s);  // w = a x + b y
hipError_t launch_cg_update(int prec, int64_t n, double alpha, const void *p, const void *q, void *x,
                            const void *r_in, void *r_out, hipStream_t s);  // x += a p; r_out = r_in - a q
hipError_t launch_jacobi_dot(int prec, int64_t n, const void *dinv, const void *r, void *z,
                             double *partial, double *out, hipStream_t s);  // z = dinv r; out = {r.z, r.r}
hipError_t launch_dot_pair(int prec, int64_t n, const void *z, const void *a, const void *b,
                           double *partial, double *out, hipStream_t s);  // out = {z.a, z.b}
hipError_t launch_cast(int64_t n, int to_prec, const void *x, void *y, hipStream_t s);
hipError_t launch_recip(int prec, int64_t n, void *x, hipStream_t s);
hipError_t launch_cheb_first(int prec, int64_t n, const void *dinv, const void *b, const void *Ax,
                             void *r, void *d, void *x, double inv_theta, hipStream_t s);
hipError_t launch_cheb_step(int prec, int64_t n, const void *dinv, void *r, const void *Ad, void *d,
                            void *x, double c1, double c2, hipStream_t s);


size_t prec_size(int prec);

}  // namespace hpmg
