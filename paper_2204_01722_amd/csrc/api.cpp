// C ABI: operator handles, argument validation, workspace carve-up and dispatch.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace {
thread_local std::string g_last_error;

inline size_t align256(size_t n) { return (n + 255) & ~size_t(255); }
inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }
}  // namespace

namespace hpmg {

int fail(int status, const std::string &msg) {
  g_last_error = msg;
  return status;
}

int hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return HPMG_ERR_HIP;
}

}  // namespace hpmg

using namespace hpmg;

struct OpExtra {
  std::vector<double> t64;
  std::vector<float> t32;
  unsigned zero = 0;
  unsigned host_flags = 0;
};

namespace {

int fill_tables(hpmg_op_s *op, OpExtra *x) {
  const int P = op->P, Q = op->Q;
  x->t64.assign(TAB_SIZE, 0.0);
  double *t = x->t64.data();
  int st = tabulate(P, Q, t + TAB_B, t + TAB_G, t + TAB_D, nullptr, t + TAB_W, nullptr);
  if (st) return st;
  for (int k = 0; k < Q * P; ++k) {
    t[TAB_BB + k] = t[TAB_B + k] * t[TAB_B + k];
    t[TAB_BG + k] = t[TAB_B + k] * t[TAB_G + k];
    t[TAB_GG + k] = t[TAB_G + k] * t[TAB_G + k];
  }
  for (int Pf = P + 1; Pf <= 6; ++Pf) {
    st = ctof_table(Pf, P, t + tab_ctof(Pf));
    if (st) return st;
  }
  x->t32.resize(TAB_SIZE);
  for (int k = 0; k < TAB_SIZE; ++k) x->t32[k] = (float)t[k];
  return HPMG_OK;
}

// Byte offsets of the workspace parts; the last entry is the total.
struct Layout {
  size_t flags, tab64, tab32, emap, scratch, csr_off, csr_inc, evec, elmat, geo, st64, st32, total;
};

Layout layout_of(const hpmg_op_s *op) {
  Layout L{};
  size_t o = 0;
  L.flags = o; o += 256;
  L.tab64 = o; o += align256(TAB_SIZE * sizeof(double));
  L.tab32 = o; o += align256(TAB_SIZE * sizeof(float));
  L.emap = o; o += align256((size_t)op->E * op->P * op->P * op->P * sizeof(uint32_t));
  L.scratch = o; o += align256(((size_t)op->E + 2 * RED_BLOCKS + 64) * sizeof(double));
  const size_t nrec = (size_t)op->E * op->P * op->P * op->P;
  L.csr_off = o; o += align256(((size_t)op->N + 1) * sizeof(int32_t));
  L.csr_inc = o; o += align256(nrec * sizeof(int32_t));
  L.evec = o; o += align256(nrec * 3 * sizeof(double));
  L.elmat = o; o += op->P == 2 ? align256((size_t)op->E * 300 * sizeof(double)) : 0;
  const size_t nq = (size_t)op->tiles * op->NQ;
  if (!op->fine) {
    L.geo = o; o += align256(nq * NGEO * sizeof(double));
    L.st64 = o; o += align256(nq * NSTATE * sizeof(double));
    L.st32 = o; o += align256(nq * NSTATE * sizeof(float));
  } else {
    L.geo = L.st64 = L.st32 = 0;
  }
  L.total = o;
  return L;
}

OpExtra *extra(hpmg_op op) { return static_cast<OpExtra *>(op->host_extra); }

int check_ready(hpmg_op op, const char *fn) {
  if (!op) return fail(HPMG_ERR_ARG, std::string(fn) + ": null operator");
  if (!op->ws) return fail(HPMG_ERR_WORKSPACE, std::string(fn) + ": workspace not bound");
  return HPMG_OK;
}
int check_prec(int prec, const char *fn) {
  if (prec != HPMG_F64 && prec != HPMG_F32) return fail(HPMG_ERR_ARG, std::string(fn) + ": bad precision");
  return HPMG_OK;
}
}  // namespace

extern "C" {

const char *hpmg_status_string(int s) {
  switch (s) {
    case HPMG_OK: return "ok";
    case HPMG_ERR_ARG: return "invalid argument";
    case HPMG_ERR_SHAPE: return "inconsistent shape";
    case HPMG_ERR_UNSUPPORTED: return "unsupported configuration";
    case HPMG_ERR_WORKSPACE: return "workspace missing or too small";
    case HPMG_ERR_HIP: return "HIP runtime error";
    case HPMG_ERR_NONPOSITIVE_J: return "non-positive Jacobian determinant";
    case HPMG_ERR_NONFINITE: return "non-finite value";
    case HPMG_ERR_BREAKDOWN: return "Krylov breakdown";
    case HPMG_ERR_NOT_CONVERGED: return "not converged";
    default: return "unknown status";
  }
}

const char *hpmg_last_error(void) { return g_last_error.c_str(); }

const char *hpmg_version(void) { return "hpmg 0.1 (gfx950)"; }

int hpmg_op_create(int P, int Q, int64_t n_elem, int64_t n_nodes, const int32_t *elem_nodes,
                   const uint8_t *mask, hpmg_op *out) {
  if (!out) return fail(HPMG_ERR_ARG, "op_create: null output");
  *out = nullptr;
  if (!supported_pq(P, Q)) return fail(HPMG_ERR_UNSUPPORTED, "op_create: (P, Q) not compiled");
  if (n_elem <= 0 || n_nodes <= 0) return fail(HPMG_ERR_SHAPE, "op_create: empty mesh");
  if (n_nodes >= MAX_NODES) return fail(HPMG_ERR_SHAPE, "op_create: too many nodes (max 2^28 - 1)");
  if (!elem_nodes) return fail(HPMG_ERR_ARG, "op_create: null element map");
  const int ET = elems_per_tile(Q);
  const int64_t tiles = (n_elem + ET - 1) / ET;
  if (tiles > 0x7fffffffLL) return fail(HPMG_ERR_SHAPE, "op_create: too many elements");
  hpmg_op_s *op = new hpmg_op_s();
  OpExtra *ex = new OpExtra();
  op->host_extra = ex;
  op->P = P;
  op->Q = Q;
  op->E = n_elem;
  op->N = n_nodes;
  op->elem_nodes = elem_nodes;
  op->mask = mask;
  op->ET = ET;
  op->NQ = ET * Q * Q * Q;
  op->NT = tile_threads(Q);
  op->tiles = tiles;
  int st = fill_tables(op, ex);
  if (st) {
    delete ex;
    delete op;
    return st;
  }
  *out = op;
  return HPMG_OK;
}

int hpmg_op_create_coarse(hpmg_op fine, int Pc, int64_t n_nodes, const int32_t *elem_nodes,
                          const uint8_t *mask, hpmg_op *out) {
  if (!out || !fine) return fail(HPMG_ERR_ARG, "op_create_coarse: null argument");
  *out = nullptr;
  if (fine->fine) return fail(HPMG_ERR_ARG, "op_create_coarse: `fine` must be a fine operator");
  if (Pc >= fine->P) return fail(HPMG_ERR_ARG, "op_create_coarse: coarse order must be lower");
  int st = hpmg_op_create(Pc, fine->Q, fine->E, n_nodes, elem_nodes, mask, out);
  if (st) return st;
  (*out)->fine = fine;
  return HPMG_OK;
}

void hpmg_op_destroy(hpmg_op op) {
  if (!op) return;
  delete extra(op);
  delete op;
}

int hpmg_op_set_material(hpmg_op op, double mu, double lambda, const double *mu_e, const double *lambda_e) {
  if (!op) return fail(HPMG_ERR_ARG, "set_material: null operator");
  if ((mu_e == nullptr) != (lambda_e == nullptr))
    return fail(HPMG_ERR_ARG, "set_material: give both per-element arrays or neither");
  if (!mu_e && !(std::isfinite(mu) && std::isfinite(lambda)))
    return fail(HPMG_ERR_ARG, "set_material: non-finite Lame parameters");
  op->mu = mu;
  op->lam = lambda;
  op->mu_e = mu_e;
  op->lam_e = lambda_e;
  return HPMG_OK;
}

int hpmg_op_workspace_bytes(hpmg_op op, size_t *bytes) {
  if (!op || !bytes) return fail(HPMG_ERR_ARG, "workspace_bytes: null argument");
  *bytes = layout_of(op).total;
  return HPMG_OK;
}

int hpmg_op_bind_workspace(hpmg_op op, void *ws, size_t bytes, void *stream) {
  if (!op || !ws) return fail(HPMG_ERR_ARG, "bind_workspace: null argument");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(HPMG_ERR_ARG, "bind_workspace: not 256-byte aligned");
  const Layout L = layout_of(op);
  if (bytes < L.total) return fail(HPMG_ERR_WORKSPACE, "bind_workspace: buffer too small");
  char *w = static_cast<char *>(ws);
  op->ws = w;
  op->ws_bytes = bytes;
  op->flags = reinterpret_cast<unsigned *>(w + L.flags);
  op->tab64 = reinterpret_cast<double *>(w + L.tab64);
  op->tab32 = reinterpret_cast<float *>(w + L.tab32);
  op->emap = reinterpret_cast<uint32_t *>(w + L.emap);
  op->scratch = reinterpret_cast<double *>(w + L.scratch);
  op->csr_off = reinterpret_cast<int32_t *>(w + L.csr_off);
  op->csr_inc = reinterpret_cast<int32_t *>(w + L.csr_inc);
  op->evec = reinterpret_cast<double *>(w + L.evec);
  op->elmat = op->P == 2 ? reinterpret_cast<double *>(w + L.elmat) : nullptr;
  op->elmat_prec = -1;
  if (!op->fine) {
    op->geo = reinterpret_cast<double *>(w + L.geo);
    op->state64 = reinterpret_cast<double *>(w + L.st64);
    op->state32 = reinterpret_cast<float *>(w + L.st32);
  }
  op->geo_ready = op->state_ready = op->state32_ready = false;
  OpExtra *x = extra(op);
  hipStream_t s = S(stream);
  HPMG_HIP(hipMemcpyAsync(op->flags, &x->zero, sizeof(unsigned), hipMemcpyHostToDevice, s));
  HPMG_HIP(hipMemcpyAsync(op->tab64, x->t64.data(), TAB_SIZE * sizeof(double), hipMemcpyHostToDevice, s));
  HPMG_HIP(hipMemcpyAsync(op->tab32, x->t32.data(), TAB_SIZE * sizeof(float), hipMemcpyHostToDevice, s));
  HPMG_HIP(launch_build_emap(*op, s));
  // The host sources of the asynchronous copies live in the handle; make sure the
  // copies have been consumed before returning so the caller may reuse the stream freely.
  HPMG_HIP(hipStreamSynchronize(s));
  unsigned fl = 0;
  HPMG_HIP(hipMemcpy(&fl, op->flags, sizeof(unsigned), hipMemcpyDeviceToHost));
  if (fl & HPMG_FLAG_BAD_INDEX) {
    op->ws = nullptr;
    return fail(HPMG_ERR_SHAPE, "bind_workspace: element map holds node ids outside [0, n_nodes)");
  }
  // Node -> element-record incidence lists (counting sort in record order, so each
  // node's contributions are always summed in the same order: the assembled result is
  // bitwise reproducible).  Built once per handle on the host.
  const int64_t P3 = (int64_t)op->P * op->P * op->P, nrec = op->E * P3;
  if (nrec >= 0x7fffffffLL) {
    op->ws = nullptr;
    return fail(HPMG_ERR_SHAPE, "bind_workspace: too many element-node records (max 2^31 - 1)");
  }
  std::vector<int32_t> en(nrec), off(op->N + 1, 0), inc(nrec);
  HPMG_HIP(hipMemcpy(en.data(), op->elem_nodes, nrec * sizeof(int32_t), hipMemcpyDeviceToHost));
  for (int64_t k = 0; k < nrec; ++k) off[en[k] + 1]++;
  for (int64_t n = 0; n < op->N; ++n) off[n + 1] += off[n];
  std::vector<int32_t> cur(off.begin(), off.end() - 1);
  for (int64_t k = 0; k < nrec; ++k) inc[cur[en[k]]++] = (int32_t)k;
  HPMG_HIP(hipMemcpy(op->csr_off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HPMG_HIP(hipMemcpy(op->csr_inc, inc.data(), inc.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HPMG_HIP(launch_mark_owners(*op, s));
  HPMG_HIP(hipStreamSynchronize(s));
  return HPMG_OK;
}

int hpmg_op_info(hpmg_op op, int64_t *info) {
  if (!op || !info) return fail(HPMG_ERR_ARG, "op_info: null argument");
  info[0] = op->P;
  info[1] = op->Q;
  info[2] = op->E;
  info[3] = op->N;
  info[4] = op->ET;
  info[5] = op->tiles;
  info[6] = op->NT;
  info[7] = op->NQ;
  return HPMG_OK;
}

int hpmg_op_state_version(hpmg_op op, uint64_t *version) {
  if (!op || !version) return fail(HPMG_ERR_ARG, "op_state_version: null argument");
  const hpmg_op_s *f = op->fine ? op->fine : op;
  *version = f->state_version;
  return HPMG_OK;
}

int hpmg_op_query_flags(hpmg_op op, void *stream, unsigned *flags) {
  int st = check_ready(op, "query_flags");
  if (st) return st;
  if (!flags) return fail(HPMG_ERR_ARG, "query_flags: null output");
  OpExtra *x = extra(op);
  hipStream_t s = S(stream);
  HPMG_HIP(hipMemcpyAsync(&x->host_flags, op->flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  HPMG_HIP(hipStreamSynchronize(s));
  HPMG_HIP(hipMemcpyAsync(op->flags, &x->zero, sizeof(unsigned), hipMemcpyHostToDevice, s));
  HPMG_HIP(hipStreamSynchronize(s));
  *flags = x->host_flags;
  return HPMG_OK;
}

int hpmg_qdata_setup(hpmg_op op, const double *coords, void *stream) {
  int st = check_ready(op, "qdata_setup");
  if (st) return st;
  if (op->fine) return fail(HPMG_ERR_ARG, "qdata_setup: coarse operators share the fine geometry");
  if (!coords) return fail(HPMG_ERR_ARG, "qdata_setup: null coordinates");
  HPMG_HIP(launch_qdata(*op, coords, S(stream)));
  op->geo_ready = true;
  return HPMG_OK;
}

int hpmg_qdata_export(hpmg_op op, double *out, void *stream) {
  int st = check_ready(op, "qdata_export");
  if (st) return st;
  if (op->fine || !op->geo_ready) return fail(HPMG_ERR_ARG, "qdata_export: no geometric factors");
  if (!out) return fail(HPMG_ERR_ARG, "qdata_export: null output");
  HPMG_HIP(launch_export_qdata(*op, out, S(stream)));
  return HPMG_OK;
}

int hpmg_residual(hpmg_op op, const double *u, double *r, int store_state, void *stream) {
  int st = check_ready(op, "residual");
  if (st) return st;
  if (op->fine) return fail(HPMG_ERR_ARG, "residual: needs a fine operator");
  if (!op->geo_ready) return fail(HPMG_ERR_ARG, "residual: call qdata_setup first");
  if (!u || !r) return fail(HPMG_ERR_ARG, "residual: null vector");
  if ((const void *)u == (const void *)r) return fail(HPMG_ERR_ARG, "residual: u and r must not alias");
  HPMG_HIP(launch_residual(*op, u, r, store_state != 0, S(stream)));
  if (store_state) {
    op->state_ready = true;
    op->state32_ready = false;
    op->state_version++;
  }
  return HPMG_OK;
}

int hpmg_state_cast_f32(hpmg_op op, void *stream) {
  int st = check_ready(op, "state_cast_f32");
  if (st) return st;
  hpmg_op_s *f = op->fine ? op->fine : op;
  if (!f->state_ready) return fail(HPMG_ERR_ARG, "state_cast_f32: no stored linearisation");
  HPMG_HIP(launch_cast_state((int64_t)f->tiles * f->NQ * NSTATE, f->state64, f->state32, S(stream)));
  f->state32_ready = true;
  return HPMG_OK;
}

int hpmg_jacobian_apply(hpmg_op op, int precision, int mode, const double *u, const void *du, void *y,
                        void *stream) {
  int st = check_ready(op, "jacobian_apply");
  if (st) return st;
  if ((st = check_prec(precision, "jacobian_apply"))) return st;
  if (!du || !y) return fail(HPMG_ERR_ARG, "jacobian_apply: null vector");
  if (du == y) return fail(HPMG_ERR_ARG, "jacobian_apply: du and y must not alias");
  const hpmg_op_s *f = op->fine ? op->fine : op;
  if (mode == HPMG_STORED) {
    if (!f->state_ready) return fail(HPMG_ERR_ARG, "jacobian_apply: no stored linearisation (residual with store_state)");
    if (precision == HPMG_F32 && !f->state32_ready)
      return fail(HPMG_ERR_ARG, "jacobian_apply: FP32 state not cast (hpmg_state_cast_f32)");
  } else if (mode == HPMG_RECOMPUTE) {
    if (op->fine) return fail(HPMG_ERR_ARG, "jacobian_apply: recompute mode needs a fine operator");
    if (!u) return fail(HPMG_ERR_ARG, "jacobian_apply: recompute mode needs u");
    if (!op->geo_ready) return fail(HPMG_ERR_ARG, "jacobian_apply: call qdata_setup first");
  } else if (mode == HPMG_INITIAL_NATIVE || mode == HPMG_INITIAL_TUNED || mode == HPMG_CURRENT_20) {
    if (op->fine) return fail(HPMG_ERR_ARG, "jacobian_apply: initial-configuration modes need a fine operator");
    if (precision != HPMG_F64) return fail(HPMG_ERR_UNSUPPORTED, "jacobian_apply: initial-configuration modes are FP64");
    if (!op->sinit_ready) return fail(HPMG_ERR_ARG, "jacobian_apply: call hpmg_state_initial first");
  } else {
    return fail(HPMG_ERR_ARG, "jacobian_apply: bad mode");
  }
  HPMG_HIP(launch_jacobian(*op, precision, mode, u, du, y, S(stream)));
  return HPMG_OK;
}

static size_t ext_layout(const hpmg_op_s *op, int64_t nf, size_t *o_rec, size_t *o_node, size_t *o_off,
                         size_t *o_inc, size_t *o_tmp) {
  const int64_t P2 = (int64_t)op->P * op->P;
  size_t o = 0;
  *o_rec = o; o += align256((size_t)nf * P2 * 3 * sizeof(double));
  *o_node = o; o += align256((size_t)nf * P2 * sizeof(int32_t));
  *o_off = o; o += align256(((size_t)op->N + 1) * sizeof(int32_t));
  *o_inc = o; o += align256((size_t)nf * P2 * sizeof(int32_t));
  *o_tmp = o; o += align256((size_t)op->N * 3 * sizeof(double));
  return o;
}

int hpmg_external_load_workspace_bytes(hpmg_op op, int64_t n_faces, size_t *bytes) {
  if (!op || !bytes || n_faces < 0) return fail(HPMG_ERR_ARG, "external_load_workspace_bytes: bad argument");
  size_t a, b, c, d, e;
  *bytes = ext_layout(op, n_faces, &a, &b, &c, &d, &e);
  return HPMG_OK;
}

int hpmg_external_load(hpmg_op op, const double *rho_g, const double *coords, int64_t n_faces,
                       const int32_t *face_elem, const int32_t *face_id, const double *traction,
                       void *workspace, size_t bytes, double *f_ext, void *stream) {
  int st = check_ready(op, "external_load");
  if (st) return st;
  if (op->fine) return fail(HPMG_ERR_ARG, "external_load: fine operators only");
  if (!f_ext || n_faces < 0) return fail(HPMG_ERR_ARG, "external_load: bad argument");
  if (n_faces > 0 && (!coords || !face_elem || !face_id || !traction))
    return fail(HPMG_ERR_ARG, "external_load: faces need coords, face lists and a traction");
  if (rho_g && !op->geo_ready) return fail(HPMG_ERR_ARG, "external_load: call qdata_setup first");
  size_t o_rec, o_node, o_off, o_inc, o_tmp;
  const size_t need = ext_layout(op, n_faces, &o_rec, &o_node, &o_off, &o_inc, &o_tmp);
  if (n_faces > 0 && (!workspace || bytes < need)) return fail(HPMG_ERR_WORKSPACE, "external_load: workspace too small");
  if (workspace && reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(HPMG_ERR_WORKSPACE, "external_load: workspace not 256-byte aligned");
  hipStream_t s = S(stream);
  const double zero[3] = {0.0, 0.0, 0.0};
  // body force (records of every element, assembled with the operator's incidence
  // lists; constrained components 0)
  HPMG_HIP(launch_body_load(*op, rho_g ? rho_g : zero, f_ext, s));
  if (n_faces == 0) return HPMG_OK;
  char *w = static_cast<char *>(workspace);
  double *rec = reinterpret_cast<double *>(w + o_rec), *tmp = reinterpret_cast<double *>(w + o_tmp);
  int32_t *rnode = reinterpret_cast<int32_t *>(w + o_node), *off = reinterpret_cast<int32_t *>(w + o_off),
          *inc = reinterpret_cast<int32_t *>(w + o_inc);
  HPMG_HIP(launch_traction_load(*op, coords, n_faces, face_elem, face_id, traction, rec, rnode, s));
  // node -> face-record incidence lists, in record order (deterministic sums)
  const int64_t nr = n_faces * op->P * op->P;
  std::vector<int32_t> nodes(nr), hoff(op->N + 1, 0), hinc(nr);
  HPMG_HIP(hipMemcpyAsync(nodes.data(), rnode, nr * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HPMG_HIP(hipStreamSynchronize(s));
  for (int64_t k = 0; k < nr; ++k) {
    if (nodes[k] < 0 || nodes[k] >= op->N) return fail(HPMG_ERR_SHAPE, "external_load: bad face element or face id");
    hoff[nodes[k] + 1]++;
  }
  for (int64_t n = 0; n < op->N; ++n) hoff[n + 1] += hoff[n];
  std::vector<int32_t> cur(hoff.begin(), hoff.end() - 1);
  for (int64_t k = 0; k < nr; ++k) hinc[cur[nodes[k]]++] = (int32_t)k;
  HPMG_HIP(hipMemcpyAsync(off, hoff.data(), hoff.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HPMG_HIP(hipMemcpyAsync(inc, hinc.data(), hinc.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HPMG_HIP(launch_assemble_csr(op->N, off, inc, rec, op->mask, tmp, s));
  HPMG_HIP(launch_axpby(HPMG_F64, 3 * op->N, 1.0, tmp, 1.0, f_ext, s));
  HPMG_HIP(hipStreamSynchronize(s));  // the host lists above must outlive the copies
  return HPMG_OK;
}

int hpmg_state_initial_bytes(hpmg_op op, size_t *bytes) {
  if (!op || !bytes) return fail(HPMG_ERR_ARG, "state_initial_bytes: null argument");
  if (op->fine) return fail(HPMG_ERR_ARG, "state_initial_bytes: fine operators only");
  *bytes = (size_t)op->tiles * NINIT * op->NQ * sizeof(double);
  return HPMG_OK;
}

int hpmg_state_initial(hpmg_op op, const double *u, void *buffer, size_t bytes, void *stream) {
  int st = check_ready(op, "state_initial");
  if (st) return st;
  if (op->fine) return fail(HPMG_ERR_ARG, "state_initial: fine operators only");
  if (!u || !buffer) return fail(HPMG_ERR_ARG, "state_initial: null argument");
  if (!op->geo_ready) return fail(HPMG_ERR_ARG, "state_initial: call qdata_setup first");
  size_t need = 0;
  hpmg_state_initial_bytes(op, &need);
  if (bytes < need) return fail(HPMG_ERR_WORKSPACE, "state_initial: buffer too small");
  if (reinterpret_cast<uintptr_t>(buffer) % 256) return fail(HPMG_ERR_WORKSPACE, "state_initial: buffer not 256-byte aligned");
  op->sinit = static_cast<double *>(buffer);
  HPMG_HIP(launch_state_initial(*op, u, S(stream)));
  op->sinit_ready = true;
  return HPMG_OK;
}

int hpmg_op_assemble_elements(hpmg_op op, int precision, void *stream) {
  int st = check_ready(op, "assemble_elements");
  if (st) return st;
  if ((st = check_prec(precision, "assemble_elements"))) return st;
  if (op->P != 2 || !op->elmat)
    return fail(HPMG_ERR_UNSUPPORTED, "assemble_elements: only for operators of order 1");
  const hpmg_op_s *src = op->fine ? op->fine : op;  // where the linearisation is stored
  if (!src->state_ready) return fail(HPMG_ERR_ARG, "assemble_elements: no stored linearisation");
  if (precision == HPMG_F32 && !src->state32_ready)
    return fail(HPMG_ERR_ARG, "assemble_elements: FP32 state not cast");
  HPMG_HIP(launch_elmat_build(*op, precision, S(stream)));
  op->elmat_prec = precision;
  op->elmat_version = src->state_version;
  return HPMG_OK;
}

int hpmg_diagonal(hpmg_op op, int precision, void *diag, void *stream) {
  int st = check_ready(op, "diagonal");
  if (st) return st;
  if ((st = check_prec(precision, "diagonal"))) return st;
  if (!diag) return fail(HPMG_ERR_ARG, "diagonal: null output");
  const hpmg_op_s *f = op->fine ? op->fine : op;
  if (!f->state_ready) return fail(HPMG_ERR_ARG, "diagonal: no stored linearisation");
  if (precision == HPMG_F32 && !f->state32_ready) return fail(HPMG_ERR_ARG, "diagonal: FP32 state not cast");
  HPMG_HIP(launch_diagonal(*op, precision, diag, S(stream)));
  return HPMG_OK;
}

static int check_pair(hpmg_op coarse, hpmg_op fine, const char *fn) {
  int st = check_ready(coarse, fn);
  if (st) return st;
  if ((st = check_ready(fine, fn))) return st;
  if (coarse->E != fine->E) return fail(HPMG_ERR_SHAPE, std::string(fn) + ": operators on different meshes");
  if (coarse->P >= fine->P) return fail(HPMG_ERR_ARG, std::string(fn) + ": coarse order must be lower");
  return HPMG_OK;
}

int hpmg_prolong_add(hpmg_op coarse, hpmg_op fine, int precision, const void *xc, void *yf, void *stream) {
  int st = check_pair(coarse, fine, "prolong_add");
  if (st) return st;
  if ((st = check_prec(precision, "prolong_add"))) return st;
  if (!xc || !yf) return fail(HPMG_ERR_ARG, "prolong_add: null vector");
  hipError_t e = launch_prolong_add(*coarse, *fine, precision, xc, yf, S(stream));
  if (e == hipErrorInvalidValue) return fail(HPMG_ERR_UNSUPPORTED, "prolong_add: order pair not compiled");
  HPMG_HIP(e);
  return HPMG_OK;
}

int hpmg_restrict(hpmg_op fine, hpmg_op coarse, int precision, const void *rf, void *rc, void *stream) {
  int st = check_pair(coarse, fine, "restrict");
  if (st) return st;
  if ((st = check_prec(precision, "restrict"))) return st;
  if (!rf || !rc) return fail(HPMG_ERR_ARG, "restrict: null vector");
  hipError_t e = launch_restrict(*fine, *coarse, precision, rf, rc, S(stream));
  if (e == hipErrorInvalidValue) return fail(HPMG_ERR_UNSUPPORTED, "restrict: order pair not compiled");
  HPMG_HIP(e);
  return HPMG_OK;
}

int hpmg_energy(hpmg_op op, const double *u, double *psi, void *stream) {
  int st = check_ready(op, "energy");
  if (st) return st;
  if (op->fine || !op->geo_ready) return fail(HPMG_ERR_ARG, "energy: needs a fine operator with geometry");
  if (!u || !psi) return fail(HPMG_ERR_ARG, "energy: null argument");
  HPMG_HIP(launch_energy(*op, u, psi, S(stream)));
  return HPMG_OK;
}

int hpmg_residual_vjp(hpmg_op op, int precision, int mode, const double *u, const void *w, void *u_bar,
                      double *mu_bar, double *lambda_bar, void *stream) {
  int st = check_ready(op, "residual_vjp");
  if (st) return st;
  if ((st = check_prec(precision, "residual_vjp"))) return st;
  if (op->fine || !op->geo_ready) return fail(HPMG_ERR_ARG, "residual_vjp: needs a fine operator with geometry");
  if (!w || !u_bar) return fail(HPMG_ERR_ARG, "residual_vjp: null vector");
  if (mode == HPMG_STORED) {
    if (!op->state_ready) return fail(HPMG_ERR_ARG, "residual_vjp: no stored linearisation");
    if (precision == HPMG_F32 && !op->state32_ready)
      return fail(HPMG_ERR_ARG, "residual_vjp: FP32 state not cast (hpmg_state_cast_f32)");
  } else if (mode == HPMG_RECOMPUTE) {
    if (!u) return fail(HPMG_ERR_ARG, "residual_vjp: recompute mode needs u");
  } else {
    return fail(HPMG_ERR_ARG, "residual_vjp: bad mode");
  }
  HPMG_HIP(launch_vjp(*op, precision, mode, u, w, u_bar, mu_bar, lambda_bar, S(stream)));
  return HPMG_OK;
}

int hpmg_vec_dot(int precision, int64_t n, const void *x, const void *y, double *out, double *scratch,
                 void *stream) {
  int st = check_prec(precision, "vec_dot");
  if (st) return st;
  if ((n > 0 && (!x || !y)) || !out || !scratch || n < 0) return fail(HPMG_ERR_ARG, "vec_dot: bad argument");
  HPMG_HIP(launch_dot(precision, n, x, y, scratch, out, S(stream)));
  return HPMG_OK;
}

}  // extern "C"

// Partial sums of hpmg_vec_dot_noalloc: one per workgroup of the reduction's fixed
// grid, every one overwritten by every call (nothing needs clearing).  Each GPU holds
// its own copy until the process ends.  In host code `scratch` names a host-side
// stand-in, not the device array: kernels get the address from scratch_address().
static __device__ __align__(256) double scratch[HPMG_NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "vec_dot_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(HPMG_ERR_UNSUPPORTED, "vec_dot_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "vec_dot_noalloc: hipGetSymbolAddress(scratch)");
    if (!p) return fail(HPMG_ERR_HIP, "vec_dot_noalloc: null address of the scratch array");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return HPMG_OK;
}
}  // namespace

extern "C" {

int hpmg_vec_dot_noalloc(int precision, int64_t n, const void *x, const void *y, double *out, void *stream) {
  int st = check_prec(precision, "vec_dot_noalloc");
  if (st) return st;
  if ((n > 0 && (!x || !y)) || !out || n < 0) return fail(HPMG_ERR_ARG, "vec_dot_noalloc: bad argument");
  // The reduction's grid is fixed, so the scratch need does not grow with n.
  static_assert(RED_BLOCKS <= HPMG_NOALLOC_SCRATCH_DOUBLES, "scratch smaller than the reduction grid");
  void *partial = nullptr;
  if ((st = scratch_address(&partial))) return st;
  HPMG_HIP(launch_dot(precision, n, x, y, static_cast<double *>(partial), out, S(stream)));
  return HPMG_OK;
}

int hpmg_vec_axpby(int precision, int64_t n, double alpha, const void *x, double beta, void *y, void *stream) {
  int st = check_prec(precision, "vec_axpby");
  if (st) return st;
  if (!x || !y || n < 0) return fail(HPMG_ERR_ARG, "vec_axpby: bad argument");
  HPMG_HIP(launch_axpby(precision, n, alpha, x, beta, y, S(stream)));
  return HPMG_OK;
}

int hpmg_vec_cast(int64_t n, int to_precision, const void *x, void *y, void *stream) {
  int st = check_prec(to_precision, "vec_cast");
  if (st) return st;
  if (!x || !y || n < 0) return fail(HPMG_ERR_ARG, "vec_cast: bad argument");
  HPMG_HIP(launch_cast(n, to_precision, x, y, S(stream)));
  return HPMG_OK;
}

}  // extern "C"
