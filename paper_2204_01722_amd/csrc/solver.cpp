// p-multigrid preconditioner, flexible CG and the Newton load-stepping driver
// (Sections III-A and III-B).  Host orchestration only: every vector operation runs
// in the library's kernels; the host reads back the few scalars that decide control
// flow (CG coefficients, norms) through a pinned buffer.
#include <algorithm>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "common.h"

using namespace hpmg;

namespace {

inline size_t align256(size_t n) { return (n + 255) & ~size_t(255); }
inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

struct Level {
  hpmg_op_s *op = nullptr;
  int64_t n = 0;  // scalars (3 * nodes)
  void *b = nullptr, *x = nullptr, *r = nullptr, *d = nullptr, *t = nullptr, *z = nullptr, *dinv = nullptr;
  double lam = 0.0;
  // rediscretised level: node map into the next finer level (nested node sets) and
  // the injected displacement its linearisation is stored at
  bool redisc = false;
  int32_t *inj = nullptr;
  double *ustate = nullptr;
  // second direction buffer of the coarsest level (assembled-operator PCG)
  void *p2 = nullptr;
};

}  // namespace

struct hpmg_mg_s {
  std::vector<Level> lv;
  hpmg_mg_params prm{};
  char *ws = nullptr;
  size_t bytes = 0;
  double *red = nullptr;     // reduction partials
  double *pq_part = nullptr; // per-workgroup partials of p.q from the coarse fused assembly
  double *scal = nullptr;    // device scalars (SC_N)
  double *host = nullptr;    // pinned host mirror (SC_N)
  // fine FP64 vectors for the Krylov and Newton drivers
  double *fr = nullptr, *fr2 = nullptr, *fz = nullptr, *fp = nullptr, *fq = nullptr;
  double *nF = nullptr, *ndu = nullptr, *nut = nullptr, *nu0 = nullptr, *nup = nullptr;
  int last_coarse_its = 0;
  int setup_done = 0;
  // Order-1 Galerkin coarsest level assembled into 3 x 3 node blocks, sliced ELL:
  // column nodes [ell_w][N] (ascending per row, -1 - n past its end) and values
  // [ell_w][9][N], rebuilt from the element matrices at every setup.
  int ell_w = 0;
  std::vector<int32_t> ell_cols_host;
  int32_t *ell_cols = nullptr;
  void *ell_vals = nullptr;
  bool ell_ready = false;
  bool ell_node_major = false;  // block layout and PCG body (coarse_block_layout)
  uint64_t ell_version = 0;  // fine state version the blocks were built from
  // counters since creation: V-cycles, coarse iterations, operator applies per level
  int64_t n_vcycles = 0, n_coarse_its = 0, n_setups = 0;
  int64_t n_applies[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

namespace {

int prec_of(const hpmg_mg_s *mg) { return mg->prm.precision; }

size_t mg_layout(hpmg_mg_s *mg, char *base) {
  size_t o = 0;
  const int prec = prec_of(mg);
  const size_t es = prec_size(prec);
  auto take = [&](size_t bytes) -> char * {
    char *p = base ? base + o : nullptr;
    o += align256(bytes);
    return p;
  };
  mg->red = reinterpret_cast<double *>(take(2 * RED_BLOCKS * sizeof(double) * 2));
  mg->scal = reinterpret_cast<double *>(take(SC_N * sizeof(double)));
  int64_t nmax = 0;
  for (const Level &L : mg->lv) nmax = std::max<int64_t>(nmax, L.n / 3);
  const int64_t nb_pq =
      std::max<int64_t>((nmax + 255) / 256, ell_pcg_blocks(mg->lv.back().n / 3, mg->ell_node_major));
  mg->pq_part = reinterpret_cast<double *>(take((size_t)(nb_pq + 1) * sizeof(double)));
  if (mg->ell_w > 0) {
    Level &C = mg->lv.back();
    const size_t nn = (size_t)(C.n / 3);
    mg->ell_cols = reinterpret_cast<int32_t *>(take((size_t)mg->ell_w * nn * sizeof(int32_t)));
    mg->ell_vals = take((size_t)mg->ell_w * 9 * nn * es);
    C.p2 = take((size_t)C.n * es);
  }
  for (Level &L : mg->lv) {
    const size_t nb = (size_t)L.n * es;
    L.b = take(nb);
    L.x = take(nb);
    L.r = take(nb);
    L.d = take(nb);
    L.t = take(nb);
    L.z = take(nb);
    L.dinv = take(nb);
  }
  for (Level &L : mg->lv) {
    if (!L.redisc) continue;
    L.inj = reinterpret_cast<int32_t *>(take((size_t)(L.n / 3) * sizeof(int32_t)));
    L.ustate = reinterpret_cast<double *>(take((size_t)L.n * sizeof(double)));
  }
  const size_t nf = (size_t)mg->lv[0].n * sizeof(double);
  mg->fr = reinterpret_cast<double *>(take(nf));
  mg->fr2 = reinterpret_cast<double *>(take(nf));
  mg->fz = reinterpret_cast<double *>(take(nf));
  mg->fp = reinterpret_cast<double *>(take(nf));
  mg->fq = reinterpret_cast<double *>(take(nf));
  mg->nF = reinterpret_cast<double *>(take(nf));
  mg->ndu = reinterpret_cast<double *>(take(nf));
  mg->nut = reinterpret_cast<double *>(take(nf));
  mg->nu0 = reinterpret_cast<double *>(take(nf));
  mg->nup = reinterpret_cast<double *>(take(nf));
  return o;
}

// Reads `count` device scalars from mg->scal (synchronises the stream).
int read_scalars(hpmg_mg_s *mg, int count, hipStream_t s) {
  HPMG_HIP(hipMemcpyAsync(mg->host, mg->scal, count * sizeof(double), hipMemcpyDeviceToHost, s));
  HPMG_HIP(hipStreamSynchronize(s));
  return HPMG_OK;
}

int apply(hpmg_mg_s *mg, const Level &L, int prec, const void *in, void *out, hipStream_t s) {
  HPMG_HIP(launch_jacobian(*L.op, prec, HPMG_STORED, nullptr, in, out, s));
  const size_t l = &L - mg->lv.data();
  if (l < 8) mg->n_applies[l]++;
  return HPMG_OK;
}

// Largest eigenvalue of a symmetric tridiagonal matrix by Sturm-sequence bisection.
double tridiag_max_eig(const std::vector<double> &a, const std::vector<double> &b) {
  const int k = (int)a.size();
  if (k == 0) return 0.0;
  double lo = a[0], hi = a[0];
  for (int i = 0; i < k; ++i) {
    double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {  // eigenvalues < x
    int c = 0;
    double q = a[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < k; ++i) {
      if (q == 0.0) q = 1e-300;
      q = a[i] - x - b[i - 1] * b[i - 1] / q;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= k)
      hi = mid;
    else
      lo = mid;
    if (hi - lo <= 1e-15 * std::max(1.0, std::fabs(hi))) break;
  }
  return hi;
}

// Jacobi-PCG on level L from x = 0 with right-hand side L.b: fixed > 0 runs exactly that
// many iterations (fewer on a breakdown, p.Ap <= 0), otherwise it stops at
// ||r|| <= rtol ||b|| or after maxit iterations.  Every scalar stays on the device and
// the stopping test runs there (after it fires, the kernels of later iterations return
// at once), so the host queues iterations in batches and reads the scalars once per
// batch: first `predict` iterations (the previous solve's count), then batches that
// double from `check`.  With alphas and betas given, the CG coefficients are read back
// (eigenvalue estimate; fixed <= PCG_RECORD) and the iterate is not formed.
int pcg_device(hpmg_mg_s *mg, Level &L, int prec, double rtol, int maxit, int fixed, int predict, int check,
               hipStream_t s, int *its_out, std::vector<double> *alphas = nullptr,
               std::vector<double> *betas = nullptr) {
  int st;
  double *sc = mg->scal;
  const bool record = alphas && betas;
  if (record && (fixed <= 0 || fixed > PCG_RECORD)) return fail(HPMG_ERR_ARG, "pcg: bad recording length");
  HPMG_HIP(launch_init_bc(prec, L.n / 3, nullptr, nullptr, L.x, s));
  HPMG_HIP(launch_waxpby(prec, L.n, 1.0, L.b, 0.0, L.b, L.r, s));
  HPMG_HIP(launch_jacobi_dot(prec, L.n, L.dinv, L.r, L.z, mg->red, sc + 2, s));  // sc[2] = rz, sc[3] = rr
  HPMG_HIP(launch_waxpby(prec, L.n, 1.0, L.z, 0.0, L.z, L.d, s));
  HPMG_HIP(launch_pcg_begin(sc, s));
  const size_t l = &L - mg->lv.data();
  const int limit = fixed > 0 ? fixed : maxit;
  const double rtol2 = fixed > 0 ? -1.0 : rtol * rtol;
  // The assembled coarsest level (when its blocks match the current linearisation)
  // takes two launches per iteration; otherwise four.
  const hpmg_op_s *src = L.op->fine ? L.op->fine : L.op;  // holder of the level's linearisation
  const bool ell = !record && l + 1 == mg->lv.size() && mg->ell_ready && mg->ell_version == src->state_version;
  const int64_t nn = L.n / 3;
  const int nb_pq = ell ? ell_pcg_blocks(nn, mg->ell_node_major) : (int)((nn + 255) / 256);
  int queued = 0, its = limit;
  int batch = fixed > 0 ? limit : std::max(check, predict), grow = check;
  while (queued < limit) {
    const int k = std::min(batch, limit - queued);
    for (int i = 0; i < k; ++i, ++queued) {
      const int parity = queued & 1;
      if (ell) {
        // Direction of iteration `queued` in (L.d, L.p2)[parity], the previous one in the other.
        void *pn = parity ? L.p2 : L.d, *po = parity ? L.d : L.p2;
        HPMG_HIP(launch_ell_pcg_apply(prec, mg->ell_node_major, nn, mg->ell_w, mg->ell_cols, mg->ell_vals, L.z, po,
                                      pn, L.t, sc,
                                      mg->red, queued, rtol2, mg->pq_part, s));
        HPMG_HIP(launch_pcg_update2(prec, L.n, sc, parity, nb_pq, mg->pq_part, pn, L.t, L.x, L.r, L.dinv, L.z,
                                    mg->red, nullptr, s));
        continue;
      }
      // Element kernel, assembly fused with p.Ap, the update (alpha from the p.Ap
      // partials) and the direction (beta from the r.z partials).
      HPMG_HIP(launch_jacobian_dot(*L.op, prec, L.d, L.t, mg->pq_part, sc + SC_STOP, s));
      HPMG_HIP(launch_pcg_update2(prec, L.n, sc, parity, nb_pq, mg->pq_part, L.d, L.t, record ? nullptr : L.x,
                                  L.r, L.dinv, L.z, mg->red, record ? sc + SC_ALPHA + queued : nullptr, s));
      HPMG_HIP(launch_pcg_dir2(prec, L.n, sc, parity, mg->red, L.z, L.d, rtol2,
                               record ? sc + SC_BETA + queued : nullptr, s));
    }
    if (fixed > 0 && !record) break;  // no read: the count is the fixed one
    // the stopping test of the last queued iteration
    if (ell) HPMG_HIP(launch_ell_pcg_apply(prec, mg->ell_node_major, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr,
                                           nullptr, sc,
                                           mg->red, queued, rtol2, nullptr, s));
    if ((st = read_scalars(mg, record ? SC_N : SC_RR0 + 1, s))) return st;
    if (mg->host[SC_STOP] != 0.0 || queued >= limit) {
      its = (int)mg->host[SC_COUNT];
      break;
    }
    batch = grow;
    grow = std::min(2 * grow, 64);
  }
  if (l < 8) mg->n_applies[l] += its;
  if (record) {
    alphas->assign(mg->host + SC_ALPHA, mg->host + SC_ALPHA + its);
    betas->assign(mg->host + SC_BETA, mg->host + SC_BETA + its);
  }
  *its_out = its;
  return HPMG_OK;
}

// Chebyshev semi-iteration for D^{-1}A on [lo, hi] * lambda_max, `degree` updates of
// L.x (Ax of the initial guess skipped when it is zero).
int chebyshev(hpmg_mg_s *mg, Level &L, int prec, bool x_zero, hipStream_t s) {
  int st;
  const double a = mg->prm.cheb_lo * L.lam, bb = mg->prm.cheb_hi * L.lam;
  const double theta = 0.5 * (bb + a), delta = 0.5 * (bb - a);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  if (x_zero) {
    HPMG_HIP(launch_cheb_first(prec, L.n, L.dinv, L.b, nullptr, L.r, L.d, L.x, 1.0 / theta, s));
  } else {
    if ((st = apply(mg, L, prec, L.x, L.t, s))) return st;
    HPMG_HIP(launch_cheb_first(prec, L.n, L.dinv, L.b, L.t, L.r, L.d, L.x, 1.0 / theta, s));
  }
  for (int k = 1; k < mg->prm.cheb_degree; ++k) {
    if ((st = apply(mg, L, prec, L.d, L.t, s))) return st;
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    HPMG_HIP(launch_cheb_step(prec, L.n, L.dinv, L.r, L.t, L.d, L.x, rho_new * rho, 2.0 * rho_new / delta, s));
    rho = rho_new;
  }
  return HPMG_OK;
}

int cycle(hpmg_mg_s *mg, int l, hipStream_t s) {
  int st;
  const int prec = prec_of(mg);
  Level &L = mg->lv[l];
  if (l + 1 == (int)mg->lv.size()) {
    int its = 0;
    st = pcg_device(mg, L, prec, mg->prm.coarse_rtol, mg->prm.coarse_maxit, mg->prm.coarse_fixed_its,
                    mg->last_coarse_its, 4, s, &its);
    mg->last_coarse_its = its;
    mg->n_coarse_its += its;
    return st;
  }
  Level &C = mg->lv[l + 1];
  if ((st = chebyshev(mg, L, prec, true, s))) return st;
  if ((st = apply(mg, L, prec, L.x, L.t, s))) return st;
  HPMG_HIP(launch_waxpby(prec, L.n, 1.0, L.b, -1.0, L.t, L.r, s));
  HPMG_HIP(launch_restrict(*L.op, *C.op, prec, L.r, C.b, s));
  if ((st = cycle(mg, l + 1, s))) return st;
  HPMG_HIP(launch_prolong_add(*C.op, *L.op, prec, C.x, L.x, s));
  return chebyshev(mg, L, prec, false, s);
}

int vcycle(hpmg_mg_s *mg, const double *r, double *z, hipStream_t s) {
  int st;
  mg->n_vcycles++;
  Level &L = mg->lv[0];
  const int prec = prec_of(mg);
  if (prec == HPMG_F64)
    HPMG_HIP(launch_waxpby(HPMG_F64, L.n, 1.0, r, 0.0, r, L.b, s));
  else
    HPMG_HIP(launch_cast(L.n, HPMG_F32, r, L.b, s));
  if ((st = cycle(mg, 0, s))) return st;
  if (prec == HPMG_F64)
    HPMG_HIP(launch_waxpby(HPMG_F64, L.n, 1.0, L.x, 0.0, L.x, z, s));
  else
    HPMG_HIP(launch_cast(L.n, HPMG_F64, L.x, z, s));
  return HPMG_OK;
}

// Sparsity of the assembled order-1 coarsest level: the nodes that share an element
// with each node, ascending.  Rows longer than ELL_MAX_W (not possible on hexahedral
// meshes whose nodes touch at most 8 elements) leave the level matrix-free.
constexpr int ELL_MAX_W = 64;
int build_ell_structure(hpmg_mg_s *mg) {
  const hpmg_op_s &C = *mg->lv.back().op;
  const int64_t nn = C.N, nrec = C.E * 8;
  std::vector<int32_t> en(nrec);
  HPMG_HIP(hipMemcpy(en.data(), C.elem_nodes, nrec * sizeof(int32_t), hipMemcpyDeviceToHost));
  std::vector<int32_t> nb((size_t)nn * ELL_MAX_W), cnt(nn, 0);
  for (int64_t e = 0; e < C.E; ++e)
    for (int a = 0; a < 8; ++a) {
      const int32_t n = en[e * 8 + a];
      if (n < 0 || n >= nn) return fail(HPMG_ERR_SHAPE, "mg_create: bad node id in the coarsest level");
      int32_t *row = nb.data() + (size_t)n * ELL_MAX_W;
      for (int b = 0; b < 8; ++b) {
        const int32_t c = en[e * 8 + b];
        bool seen = false;
        for (int k = 0; k < cnt[n] && !seen; ++k) seen = row[k] == c;
        if (seen) continue;
        if (cnt[n] == ELL_MAX_W) return HPMG_OK;  // too wide: stay matrix-free
        row[cnt[n]++] = c;
      }
    }
  int w = 0;
  for (int64_t n = 0; n < nn; ++n) {
    std::sort(nb.begin() + n * ELL_MAX_W, nb.begin() + n * ELL_MAX_W + cnt[n]);
    w = std::max(w, cnt[n]);
  }
  // padding slots hold -1 - n: the node itself, with a zero block
  mg->ell_cols_host.resize((size_t)w * nn);
  for (int64_t n = 0; n < nn; ++n)
    for (int k = 0; k < w; ++k)
      mg->ell_cols_host[(size_t)k * nn + n] = k < cnt[n] ? nb[(size_t)n * ELL_MAX_W + k] : (int32_t)(-1 - n);
  mg->ell_w = w;
  return HPMG_OK;
}

int mg_check(hpmg_mg_s *mg, const char *fn) {
  if (!mg) return fail(HPMG_ERR_ARG, std::string(fn) + ": null multigrid handle");
  if (!mg->ws) return fail(HPMG_ERR_WORKSPACE, std::string(fn) + ": workspace not bound");
  return HPMG_OK;
}

bool has_redisc(const hpmg_mg_s *mg) { return mg->lv.size() > 1 && mg->lv[1].redisc; }

// Stores the linearisation of every rediscretised level at the injection of u.
int set_state(hpmg_mg_s *mg, const double *u, hipStream_t s) {
  const double *src = u;
  for (size_t l = 1; l < mg->lv.size(); ++l) {
    Level &L = mg->lv[l];
    if (!L.redisc) continue;
    HPMG_HIP(launch_inject(L.n / 3, L.inj, src, L.ustate, s));
    hpmg_op_s *o = L.op;
    if (!o->geo_ready) return fail(HPMG_ERR_ARG, "mg_set_state: call qdata_setup on every rediscretised level");
    HPMG_HIP(launch_residual(*o, L.ustate, mg->fr, true, s));
    o->state_version++;
    o->state_ready = true;
    o->state32_ready = false;
    unsigned fl = 0;
    int st = hpmg_op_query_flags(o, s, &fl);
    if (st) return st;
    if (fl & (HPMG_FLAG_NONPOSITIVE_J | HPMG_FLAG_NONFINITE))
      return fail(HPMG_ERR_NONPOSITIVE_J, "mg_set_state: inverted element on a rediscretised level");
    src = L.ustate;
  }
  return HPMG_OK;
}

int do_setup(hpmg_mg_s *mg, const double *const *seeds, hipStream_t s) {
  int st;
  const int prec = prec_of(mg);
  for (Level &L : mg->lv) {
    hpmg_op_s *o = L.op;
    if (o->fine) continue;  // Galerkin coarse level: shares the fine state
    if (!o->state_ready)
      return fail(HPMG_ERR_ARG, L.redisc ? "mg_setup: rediscretised level without state (hpmg_mg_set_state)"
                                         : "mg_setup: no stored linearisation on the fine operator");
    if (prec == HPMG_F32) {
      HPMG_HIP(launch_cast_state((int64_t)o->tiles * o->NQ * NSTATE, o->state64, o->state32, s));
      o->state32_ready = true;
    }
  }
  for (Level &L : mg->lv) {
    HPMG_HIP(launch_diagonal(*L.op, prec, L.dinv, s));
    HPMG_HIP(launch_recip(prec, L.n, L.dinv, s));
  }
  Level &Lc = mg->lv.back();
  mg->ell_ready = false;
  if (mg->prm.coarse_element_matrices && Lc.op->P == 2 && Lc.op->elmat && Lc.op->fine) {
    const hpmg_op_s *src = Lc.op->fine;
    HPMG_HIP(launch_elmat_build(*Lc.op, prec, s));
    Lc.op->elmat_prec = prec;
    Lc.op->elmat_version = src->state_version;
    if (mg->ell_w > 0) {
      HPMG_HIP(launch_ell_build(*Lc.op, prec, mg->ell_node_major, mg->ell_w, mg->ell_cols, mg->ell_vals, s));
      mg->ell_ready = true;
      mg->ell_version = src->state_version;
    }
  }
  for (size_t l = 0; l + 1 < mg->lv.size(); ++l) {
    Level &L = mg->lv[l];
    if (prec == HPMG_F64)
      HPMG_HIP(launch_waxpby(HPMG_F64, L.n, 1.0, seeds[l], 0.0, seeds[l], L.b, s));
    else
      HPMG_HIP(launch_cast(L.n, HPMG_F32, seeds[l], L.b, s));
    std::vector<double> al, be;
    int its = 0;
    if ((st = pcg_device(mg, L, prec, 0.0, 0, mg->prm.lanczos_its, 0, 0, s, &its, &al, &be))) return st;
    if (al.empty()) return fail(HPMG_ERR_BREAKDOWN, "mg_setup: eigenvalue estimate broke down");
    std::vector<double> diag(al.size()), off(al.size() > 1 ? al.size() - 1 : 0);
    for (size_t j = 0; j < al.size(); ++j) {
      diag[j] = 1.0 / al[j] + (j > 0 ? be[j - 1] / al[j - 1] : 0.0);
      if (j + 1 < al.size()) off[j] = std::sqrt(be[j]) / al[j];
    }
    L.lam = tridiag_max_eig(diag, off);
    if (!(L.lam > 0.0) || !std::isfinite(L.lam)) return fail(HPMG_ERR_BREAKDOWN, "mg_setup: bad lambda_max");
  }
  mg->setup_done = 1;
  mg->n_setups++;
  return HPMG_OK;
}

// natural: stop on the preconditioned (natural) norm sqrt(r^T M^-1 r) relative to its
// start value instead of the 2-norm of r; the V-cycle of an iteration's new residual is
// then applied before the test (it is the next iteration's anyway).
int do_fcg(hpmg_op fine, hpmg_mg_s *mg, const double *b, double *x, double rtol, int maxit, int *its_out,
           double *rel_out, hipStream_t s, bool natural) {
  int st;
  const int64_t n = mg->lv[0].n;
  double *sc = mg->scal;
  double *r = mg->fr, *rn = mg->fr2, *z = mg->fz, *p = mg->fp, *q = mg->fq;
  *its_out = 0;
  *rel_out = 0.0;
  HPMG_HIP(launch_jacobian(*fine, HPMG_F64, HPMG_STORED, nullptr, x, q, s));
  HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, b, -1.0, q, r, s));
  HPMG_HIP(launch_dot(HPMG_F64, n, r, r, mg->red, sc, s));
  if ((st = read_scalars(mg, 1, s))) return st;
  const double r0 = std::sqrt(mg->host[0]);
  if (r0 == 0.0) return HPMG_OK;
  if ((st = vcycle(mg, r, z, s))) return st;
  HPMG_HIP(launch_dot(HPMG_F64, n, r, z, mg->red, sc + FCG_RZ, s));
  HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, z, 0.0, z, p, s));
  double nat0 = 0.0;
  if (natural) {
    if ((st = read_scalars(mg, FCG_RZ + 1, s))) return st;
    nat0 = std::sqrt(std::fabs(mg->host[FCG_RZ]));
    if (!(nat0 > 0.0)) return HPMG_OK;
  }
  // alpha and beta are formed on the device from the dot products; the host reads the
  // scalars once per iteration, for the convergence and breakdown tests.
  int its = 0;
  double rel = 1.0;
  while (its < maxit) {
    HPMG_HIP(launch_jacobian(*fine, HPMG_F64, HPMG_STORED, nullptr, p, q, s));
    HPMG_HIP(launch_dot(HPMG_F64, n, p, q, mg->red, sc + FCG_PQ, s));
    HPMG_HIP(launch_fcg_update(n, sc, its, p, q, x, r, rn, mg->red, s));
    double *zn = z;  // where M^-1 rn goes
    if (natural) {
      // M^-1 rn and its dot with rn (the natural norm squared) and r, before the tests;
      // into q's buffer (q is spent once x and rn are updated), so that z still holds
      // M^-1 r for the breakdown path
      zn = q;
      if ((st = vcycle(mg, rn, zn, s))) return st;
      HPMG_HIP(launch_dot_pair(HPMG_F64, n, zn, rn, r, mg->red, sc + FCG_ZRN, s));
    }
    if ((st = read_scalars(mg, FCG_RZ + 2, s))) return st;
    if (mg->host[FCG_BRK] != 0.0) {
      // Negative curvature (or a non-finite preconditioned residual): stop here, x as it
      // was.  Before the first step the preconditioned residual is returned instead, so a
      // caller can still search along a descent direction.
      if (its == 0 && std::isfinite(mg->host[FCG_RZ])) HPMG_HIP(launch_axpby(HPMG_F64, n, 1.0, z, 1.0, x, s));
      *its_out = its;
      *rel_out = rel;
      return fail(HPMG_ERR_BREAKDOWN, "fcg: p^T A p <= 0");
    }
    ++its;
    rel = natural ? std::sqrt(std::fabs(mg->host[FCG_ZRN])) / nat0 : std::sqrt(mg->host[FCG_RR]) / r0;
    if (rel <= rtol) break;
    if (!natural) {
      if ((st = vcycle(mg, rn, z, s))) return st;
      HPMG_HIP(launch_dot_pair(HPMG_F64, n, z, rn, r, mg->red, sc + FCG_ZRN, s));  // z.rn, z.r
    }
    HPMG_HIP(launch_fcg_dir(n, sc, its - 1, zn, p, s));
    std::swap(r, rn);
    if (natural) std::swap(z, q);
  }
  *its_out = its;
  *rel_out = rel;
  if (rel > rtol) return fail(HPMG_ERR_NOT_CONVERGED, "fcg: iteration limit reached");
  return HPMG_OK;
}

}  // namespace

extern "C" {

void hpmg_mg_default_params(hpmg_mg_params *p) {
  if (!p) return;
  p->cheb_degree = 3;
  p->cheb_lo = 0.1;
  p->cheb_hi = 1.1;
  p->lanczos_its = 10;
  p->coarse_rtol = 1e-3;
  p->coarse_maxit = 10000;
  p->coarse_fixed_its = 0;
  p->precision = HPMG_F64;
  p->coarse_element_matrices = 1;
  p->coarse_block_layout = -1;
}

int hpmg_mg_create(const hpmg_op *levels, int n_levels, const hpmg_mg_params *params, hpmg_mg *out) {
  if (!out || !levels || !params) return fail(HPMG_ERR_ARG, "mg_create: null argument");
  *out = nullptr;
  if (n_levels < 2) return fail(HPMG_ERR_ARG, "mg_create: need at least two levels");
  if (params->precision != HPMG_F64 && params->precision != HPMG_F32)
    return fail(HPMG_ERR_ARG, "mg_create: bad precision");
  if (params->cheb_degree < 1 || !(params->cheb_lo > 0.0) || !(params->cheb_hi > params->cheb_lo) ||
      params->lanczos_its < 1 || params->lanczos_its > PCG_RECORD || params->coarse_maxit < 1)
    return fail(HPMG_ERR_ARG, "mg_create: bad smoother or coarse-solver parameters");
  if (params->coarse_block_layout < -1 || params->coarse_block_layout > 1)
    return fail(HPMG_ERR_ARG, "mg_create: coarse_block_layout must be -1, 0 or 1");
  const hpmg_op_s *f = levels[0];
  if (!f || f->fine) return fail(HPMG_ERR_ARG, "mg_create: levels[0] must be a fine operator");
  // Coarse levels are either all Galerkin (coarse operators of levels[0], sharing its
  // state) or all rediscretised (operators of their own order and quadrature on the
  // same elements, their state stored at the injected field by hpmg_mg_set_state).
  const bool redisc = levels[1] && !levels[1]->fine;
  for (int l = 1; l < n_levels; ++l) {
    if (!levels[l]) return fail(HPMG_ERR_ARG, "mg_create: null level");
    if (redisc ? (levels[l]->fine != nullptr) : (levels[l]->fine != f))
      return fail(HPMG_ERR_ARG, "mg_create: coarse levels must all be coarse operators of levels[0] or all "
                                "stand-alone (rediscretised) operators");
    if (levels[l]->P >= levels[l - 1]->P) return fail(HPMG_ERR_ARG, "mg_create: orders must decrease");
    if (redisc) {
      if (levels[l]->E != f->E) return fail(HPMG_ERR_SHAPE, "mg_create: rediscretised levels need the same elements");
      const int Pf = levels[l - 1]->P, Pc = levels[l]->P;
      double gf[16], gc[16];
      if (tabulate(Pf, Pf, nullptr, nullptr, nullptr, nullptr, nullptr, gf) ||
          tabulate(Pc, Pc, nullptr, nullptr, nullptr, nullptr, nullptr, gc))
        return fail(HPMG_ERR_ARG, "mg_create: bad order");
      bool nested = (Pf - 1) % (Pc - 1) == 0;
      const int st = nested ? (Pf - 1) / (Pc - 1) : 1;
      for (int a = 0; nested && a < Pc; ++a) nested = std::fabs(gf[st * a] - gc[a]) < 1e-13;
      if (!nested)
        return fail(HPMG_ERR_UNSUPPORTED, "mg_create: rediscretised levels need nested node sets (order "
                                          "p_c = 1, or p_c = 2 below an even order)");
    }
  }
  hpmg_mg_s *mg = new hpmg_mg_s();
  mg->prm = *params;
  for (int l = 0; l < n_levels; ++l) {
    Level L;
    L.op = levels[l];
    L.n = 3 * levels[l]->N;
    L.redisc = l > 0 && redisc;
    mg->lv.push_back(L);
  }
  // Galerkin order-1 coarsest level only: a rediscretised one on its own 2^3 Gauss points
  // is cheaper matrix-free than as assembled blocks (measured)
  if (!redisc && params->coarse_element_matrices && mg->lv.back().op->P == 2) {
    const int64_t nn = mg->lv.back().n / 3;
    mg->ell_node_major = params->coarse_block_layout < 0 ? nn >= ELL_NODE_MAJOR_MIN : params->coarse_block_layout == 1;
    const int st = build_ell_structure(mg);
    if (st) {
      delete mg;
      return st;
    }
  }
  if (hipHostMalloc((void **)&mg->host, SC_N * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    delete mg;
    return fail(HPMG_ERR_HIP, "mg_create: pinned host buffer");
  }
  *out = mg;
  return HPMG_OK;
}

void hpmg_mg_destroy(hpmg_mg mg) {
  if (!mg) return;
  if (mg->host) (void)hipHostFree(mg->host);
  delete mg;
}

int hpmg_mg_workspace_bytes(hpmg_mg mg, size_t *bytes) {
  if (!mg || !bytes) return fail(HPMG_ERR_ARG, "mg_workspace_bytes: null argument");
  *bytes = mg_layout(mg, nullptr);
  return HPMG_OK;
}

int hpmg_mg_bind_workspace(hpmg_mg mg, void *ws, size_t bytes) {
  if (!mg || !ws) return fail(HPMG_ERR_ARG, "mg_bind_workspace: null argument");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(HPMG_ERR_ARG, "mg_bind_workspace: not 256-byte aligned");
  if (bytes < mg_layout(mg, nullptr)) return fail(HPMG_ERR_WORKSPACE, "mg_bind_workspace: buffer too small");
  mg->ws = static_cast<char *>(ws);
  mg->bytes = bytes;
  mg_layout(mg, mg->ws);
  mg->setup_done = 0;
  mg->ell_ready = false;
  if (mg->ell_w > 0)
    HPMG_HIP(hipMemcpy(mg->ell_cols, mg->ell_cols_host.data(), mg->ell_cols_host.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice));
  // Injection maps of rediscretised levels: coarse local node (a1, a2, a3) of an
  // element sits at fine local node (s a1, s a2, s a3), s = (Pf - 1) / (Pc - 1).
  for (size_t l = 1; l < mg->lv.size(); ++l) {
    Level &L = mg->lv[l];
    if (!L.redisc) continue;
    const hpmg_op_s &F = *mg->lv[l - 1].op, &Cc = *L.op;
    const int Pf = F.P, Pc = Cc.P, st = (Pf - 1) / (Pc - 1);
    const int64_t nf = F.E * Pf * Pf * Pf, nc = Cc.E * Pc * Pc * Pc;
    std::vector<int32_t> ef(nf), ec(nc), map(Cc.N, -1);
    HPMG_HIP(hipMemcpy(ef.data(), F.elem_nodes, nf * sizeof(int32_t), hipMemcpyDeviceToHost));
    HPMG_HIP(hipMemcpy(ec.data(), Cc.elem_nodes, nc * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int64_t e = 0; e < Cc.E; ++e)
      for (int a3 = 0; a3 < Pc; ++a3)
        for (int a2 = 0; a2 < Pc; ++a2)
          for (int a1 = 0; a1 < Pc; ++a1) {
            const int32_t c = ec[e * Pc * Pc * Pc + a1 + Pc * (a2 + Pc * a3)];
            const int32_t fn = ef[e * Pf * Pf * Pf + st * a1 + Pf * (st * a2 + Pf * st * a3)];
            if (c < 0 || c >= Cc.N || fn < 0 || fn >= F.N) return fail(HPMG_ERR_SHAPE, "mg_bind_workspace: bad node id");
            if (map[c] >= 0 && map[c] != fn)
              return fail(HPMG_ERR_SHAPE, "mg_bind_workspace: coarse node maps to two fine nodes");
            map[c] = fn;
          }
    for (int64_t c = 0; c < Cc.N; ++c)
      if (map[c] < 0) return fail(HPMG_ERR_SHAPE, "mg_bind_workspace: coarse node in no element");
    HPMG_HIP(hipMemcpy(L.inj, map.data(), map.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  }
  return HPMG_OK;
}

int hpmg_mg_set_state(hpmg_mg mg, const double *u, void *stream) {
  int st = mg_check(mg, "mg_set_state");
  if (st) return st;
  if (!u) return fail(HPMG_ERR_ARG, "mg_set_state: null u");
  if (!has_redisc(mg)) return HPMG_OK;
  return set_state(mg, u, S(stream));
}

int hpmg_mg_setup(hpmg_mg mg, const double *const *seeds, void *stream) {
  int st = mg_check(mg, "mg_setup");
  if (st) return st;
  if (!seeds) return fail(HPMG_ERR_ARG, "mg_setup: null seeds");
  for (size_t l = 0; l + 1 < mg->lv.size(); ++l)
    if (!seeds[l]) return fail(HPMG_ERR_ARG, "mg_setup: null seed vector");
  for (const Level &L : mg->lv)
    if (!L.op->ws) return fail(HPMG_ERR_WORKSPACE, "mg_setup: level operator without workspace");
  return do_setup(mg, seeds, S(stream));
}

int hpmg_mg_vcycle(hpmg_mg mg, const double *r, double *z, void *stream) {
  int st = mg_check(mg, "mg_vcycle");
  if (st) return st;
  if (!mg->setup_done) return fail(HPMG_ERR_ARG, "mg_vcycle: call mg_setup first");
  if (!r || !z) return fail(HPMG_ERR_ARG, "mg_vcycle: null vector");
  return vcycle(mg, r, z, S(stream));
}

int hpmg_mg_info(hpmg_mg mg, int level, double *lambda_max, int *last_coarse_its) {
  if (!mg) return fail(HPMG_ERR_ARG, "mg_info: null handle");
  if (level < 0 || level >= (int)mg->lv.size()) return fail(HPMG_ERR_ARG, "mg_info: bad level");
  if (lambda_max) *lambda_max = mg->lv[level].lam;
  if (last_coarse_its) *last_coarse_its = mg->last_coarse_its;
  return HPMG_OK;
}

int hpmg_mg_stats(hpmg_mg mg, int64_t *out) {
  if (!mg || !out) return fail(HPMG_ERR_ARG, "mg_stats: null argument");
  out[0] = mg->n_vcycles;
  out[1] = mg->n_coarse_its;
  out[2] = mg->n_setups;
  for (int l = 0; l < 8; ++l) out[3 + l] = mg->n_applies[l];
  return HPMG_OK;
}

int hpmg_fcg_solve(hpmg_op fine, hpmg_mg mg, const double *b, double *x, double rtol, int maxit, int *its,
                   double *relres, void *stream) {
  int st = mg_check(mg, "fcg_solve");
  if (st) return st;
  if (!fine || fine != mg->lv[0].op) return fail(HPMG_ERR_ARG, "fcg_solve: operator is not the mg fine level");
  if (!b || !x || !its || !relres) return fail(HPMG_ERR_ARG, "fcg_solve: null argument");
  if (!mg->setup_done) return fail(HPMG_ERR_ARG, "fcg_solve: call mg_setup first");
  if (!(rtol > 0.0) || maxit < 1) return fail(HPMG_ERR_ARG, "fcg_solve: bad tolerance");
  return do_fcg(fine, mg, b, x, rtol, maxit, its, relres, S(stream), false);
}

void hpmg_newton_default_params(hpmg_newton_params *p) {
  if (!p) return;
  p->rtol = 1e-8;
  p->max_newton = 20;
  p->lin_rtol = 1e-3;
  p->lin_maxit = 500;
  p->line_search = 1;
  p->monitor = 0;
  p->max_total_newton = 200;
  p->max_total_krylov = 20000;
  p->predictor = 1;
  p->lin_norm = 0;
}

// Iteration budget of a whole Newton solve (every load step and retry together).
struct NewtonBudget {
  int newton_left, krylov_left;
  bool exhausted = false;
};

// Stores the linearisation at u (residual with state) and returns ||F(u)||.
static int store_state(hpmg_op fine, hpmg_mg_s *mg, const double *u, hipStream_t s, double *fnorm) {
  int st;
  const int64_t n = mg->lv[0].n;
  HPMG_HIP(launch_residual(*fine, u, mg->nF, true, s));
  fine->state_version++;
  fine->state_ready = true;
  fine->state32_ready = false;
  HPMG_HIP(launch_dot(HPMG_F64, n, mg->nF, mg->nF, mg->red, mg->scal, s));
  if ((st = read_scalars(mg, 1, s))) return st;
  *fnorm = std::sqrt(mg->host[0]);
  return HPMG_OK;
}

// Newton solve at one load level (Section III-A).  On entry u holds the start of the
// increment.  With state_at_start the stored linearisation belongs to u (a secant-
// extrapolated start); otherwise u is the previous converged state plus the lifted load
// increment and the stored linearisation belongs to that previous state (saved in nu0):
// the first correction is taken with that tangent (an Euler predictor for the
// increment).  Later corrections use the tangent at the current iterate.  Every
// accepted point is checked for inverted elements and non-finite values; the step is
// halved (at most 6 times) until it passes.  Returns HPMG_OK on convergence, else an
// error that tells the caller to cut the increment.
static int newton_at_load(hpmg_op fine, hpmg_mg_s *mg, double *u, const double *f_ext,
                          const hpmg_newton_params *prm, const double *const *seeds, void *stream, double load,
                          bool state_at_start, NewtonBudget *budget, int *its_out, int *lin_out, double *rel_out) {
  int st;
  hipStream_t s = S(stream);
  const int64_t n = mg->lv[0].n;
  double *F = mg->nF, *du = mg->ndu, *ut = mg->nut;
  *its_out = 0;
  *rel_out = 0.0;
  HPMG_HIP(launch_residual(*fine, u, F, false, s));
  if (f_ext) HPMG_HIP(launch_axpby(HPMG_F64, n, -load, f_ext, 1.0, F, s));
  HPMG_HIP(launch_dot(HPMG_F64, n, F, F, mg->red, mg->scal, s));
  if ((st = read_scalars(mg, 1, s))) return st;
  const double f0 = std::sqrt(mg->host[0]);
  unsigned fl = 0;
  if ((st = hpmg_op_query_flags(fine, stream, &fl))) return st;
  if (fl & HPMG_FLAG_NONPOSITIVE_J) return fail(HPMG_ERR_NONPOSITIVE_J, "newton: inverted element");
  if ((fl & HPMG_FLAG_NONFINITE) || !std::isfinite(f0)) return fail(HPMG_ERR_NONFINITE, "newton: non-finite residual");
  double fn = f0;
  int its = 0;
  while (f0 > 0.0 && !(fn <= prm->rtol * f0)) {
    if (its >= prm->max_newton) return fail(HPMG_ERR_NOT_CONVERGED, "newton: iteration limit");
    if (budget->newton_left <= 0 || budget->krylov_left <= 0) {
      budget->exhausted = true;
      return fail(HPMG_ERR_NOT_CONVERGED, "newton_solve: total iteration budget spent");
    }
    budget->newton_left--;
    // the fine state belongs to the previous converged point in the predictor
    // iteration (saved in nu0), to u afterwards
    if (has_redisc(mg) && (st = set_state(mg, its == 0 && !state_at_start ? mg->nu0 : u, s))) return st;
    if ((st = do_setup(mg, seeds, s))) return st;
    HPMG_HIP(launch_waxpby(HPMG_F64, n, -1.0, F, 0.0, F, ut, s));
    HPMG_HIP(launch_init_bc(HPMG_F64, n / 3, nullptr, nullptr, du, s));
    int lits = 0;
    double lrel = 0.0;
    st = do_fcg(fine, mg, ut, du, prm->lin_rtol, std::min(prm->lin_maxit, budget->krylov_left), &lits, &lrel, s,
                prm->lin_norm == 1);
    *lin_out += lits;
    budget->krylov_left -= lits;
    if (st && st != HPMG_ERR_NOT_CONVERGED && st != HPMG_ERR_BREAKDOWN) return st;
    const int lin_st = st;
    double alpha = 1.0;
    HPMG_HIP(launch_dot(HPMG_F64, n, F, du, mg->red, mg->scal, s));
    if ((st = read_scalars(mg, 1, s))) return st;
    const double g0 = mg->host[0];
    if (!(g0 < 0.0)) return fail(HPMG_ERR_BREAKDOWN, "newton: no descent direction");
    if (prm->line_search) {
      // g(a) = F(u + a du)^T du; one secant step from a = 0 and a = 1.
      HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, u, 1.0, du, ut, s));
      HPMG_HIP(launch_residual(*fine, ut, mg->fq, false, s));
      if (f_ext) HPMG_HIP(launch_axpby(HPMG_F64, n, -load, f_ext, 1.0, mg->fq, s));
      HPMG_HIP(launch_dot(HPMG_F64, n, mg->fq, du, mg->red, mg->scal, s));
      if ((st = read_scalars(mg, 1, s))) return st;
      const double g1 = mg->host[0];
      unsigned fl2 = 0;
      if ((st = hpmg_op_query_flags(fine, stream, &fl2))) return st;  // clears the trial point's flags
      // Secant root of g between 0 and 1 when its secant slope is positive; else 1.
      if (std::isfinite(g1) && !fl2 && g1 - g0 > 0.0) alpha = std::min(1.5, std::max(0.1, g0 / (g0 - g1)));
      else if (!std::isfinite(g1) || fl2) alpha = 0.5;
    }
    // Accept u + alpha du, halving alpha while the point has an inverted element or a
    // non-finite residual.  The state stored by the last evaluation belongs to the
    // accepted point.
    bool ok = false;
    for (int bt = 0; bt < 7; ++bt) {
      HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, u, alpha, du, ut, s));
      HPMG_HIP(launch_residual(*fine, ut, F, true, s));
      fine->state_version++;
      fine->state_ready = true;
      fine->state32_ready = false;
      if (f_ext) HPMG_HIP(launch_axpby(HPMG_F64, n, -load, f_ext, 1.0, F, s));
      HPMG_HIP(launch_dot(HPMG_F64, n, F, F, mg->red, mg->scal, s));
      if ((st = read_scalars(mg, 1, s))) return st;
      fn = std::sqrt(mg->host[0]);
      unsigned fl3 = 0;
      if ((st = hpmg_op_query_flags(fine, stream, &fl3))) return st;
      ok = std::isfinite(fn) && !(fl3 & (HPMG_FLAG_NONPOSITIVE_J | HPMG_FLAG_NONFINITE));
      if (ok) break;
      alpha *= 0.5;
    }
    if (!ok) return fail(HPMG_ERR_NONPOSITIVE_J, "newton: no admissible step length");
    HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, ut, 0.0, ut, u, s));
    ++its;
    *its_out = its;
    *rel_out = fn / f0;
    if (prm->monitor)
      std::fprintf(stderr, "[newton] load %.6f it %d rel %.3e fcg %d (%s, rel %.2e) alpha %.3f\n", load, its,
                   fn / f0, lits, lin_st == HPMG_OK ? "ok" : lin_st == HPMG_ERR_BREAKDOWN ? "breakdown" : "maxit",
                   lrel, alpha);
  }
  return HPMG_OK;
}

int hpmg_newton_solve(hpmg_op fine, hpmg_mg mg, double *u, const double *lift, const double *f_ext, int n_steps,
                      const hpmg_newton_params *prm, const double *const *seeds, double *stats, void *stream) {
  // parameters first: nothing behind the handles is touched before they pass
  if (!u || !lift || !prm || !seeds || !stats) return fail(HPMG_ERR_ARG, "newton_solve: null argument");
  if (n_steps < 1 || n_steps > 60) return fail(HPMG_ERR_ARG, "newton_solve: 1 <= n_steps <= 60");
  if (prm->max_total_newton < 1 || prm->max_total_krylov < 1)
    return fail(HPMG_ERR_ARG, "newton_solve: the total iteration budgets must be positive");
  if (prm->max_newton < 1 || prm->lin_maxit < 1 || !(prm->rtol > 0.0) || !(prm->lin_rtol > 0.0))
    return fail(HPMG_ERR_ARG, "newton_solve: iteration limits and tolerances must be positive");
  if (prm->lin_norm != 0 && prm->lin_norm != 1)
    return fail(HPMG_ERR_ARG, "newton_solve: lin_norm must be 0 (2-norm) or 1 (natural norm)");
  int st = mg_check(mg, "newton_solve");
  if (st) return st;
  if (!fine || fine != mg->lv[0].op) return fail(HPMG_ERR_ARG, "newton_solve: operator is not the mg fine level");
  if (!fine->geo_ready) return fail(HPMG_ERR_ARG, "newton_solve: call qdata_setup first");
  hipStream_t s = S(stream);
  const int64_t n = mg->lv[0].n;
  for (int k = 0; k < 4 + n_steps; ++k) stats[k] = 0.0;
  int total_newton = 0, total_lin = 0, cuts = 0;
  NewtonBudget budget{prm->max_total_newton, prm->max_total_krylov};
  // Secant predictor: once two converged load levels are known (nup, then u), a new
  // increment starts from their linear extrapolation, which carries the previous
  // increment's deformation pattern (for stiff inclusions: the soft matrix takes the
  // compression) instead of the affine lifting; constrained components still receive
  // exactly the prescribed increment.
  bool have_prev = false;
  double prev_inc = 0.0;
  double final_rel = 0.0;
  // Load increments of 1/n_steps; an increment whose Newton solve fails is retried from
  // the previous converged state in halves (at most 6 halvings in a row); after a
  // success the increment doubles again, up to the full step.
  bool state_at_u = false;  // does the stored linearisation belong to u?
  for (int step = 0; step < n_steps; ++step) {
    double done = 0.0, dt = 1.0;
    int halvings = 0;
    while (done < 1.0 - 1e-12) {
      const double inc = std::min(dt, 1.0 - done);
      if (!state_at_u) {
        double f_prev = 0.0;
        if ((st = store_state(fine, mg, u, s, &f_prev))) return st;
        unsigned fl = 0;
        if ((st = hpmg_op_query_flags(fine, stream, &fl))) return st;
        if (fl & (HPMG_FLAG_NONPOSITIVE_J | HPMG_FLAG_NONFINITE) || !std::isfinite(f_prev))
          return fail(HPMG_ERR_NONPOSITIVE_J, "newton_solve: the starting state has an inverted element");
        state_at_u = true;
      }
      HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, u, 0.0, u, mg->nu0, s));
      bool extrapolated = false;
      if (prm->predictor && have_prev) {
        const double r = inc / prev_inc;
        HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0 + r, mg->nu0, -r, mg->nup, u, s));
        double f_start = 0.0;
        if ((st = store_state(fine, mg, u, s, &f_start))) return st;
        unsigned fl = 0;
        if ((st = hpmg_op_query_flags(fine, stream, &fl))) return st;
        extrapolated = std::isfinite(f_start) && !(fl & (HPMG_FLAG_NONPOSITIVE_J | HPMG_FLAG_NONFINITE));
        if (!extrapolated) {  // inadmissible start: back to the lifted start from nu0
          HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, mg->nu0, 0.0, mg->nu0, u, s));
          if ((st = store_state(fine, mg, u, s, &f_start))) return st;
          if ((st = hpmg_op_query_flags(fine, stream, &fl))) return st;
        }
        state_at_u = true;
      }
      if (!extrapolated) HPMG_HIP(launch_axpby(HPMG_F64, n, inc / n_steps, lift, 1.0, u, s));
      if (prm->monitor)
        std::fprintf(stderr, "[newton] load %.6f start: %s\n", (step + done + inc) / n_steps,
                     extrapolated ? "secant extrapolation" : "lifted increment");
      int its = 0;
      double rel = 0.0;
      st = newton_at_load(fine, mg, u, f_ext, prm, seeds, stream, (step + done + inc) / n_steps, extrapolated,
                          &budget, &its, &total_lin, &rel);
      if (st && prm->monitor)
        std::fprintf(stderr, "[newton] load %.6f failed (%s); halving the increment\n", (step + done + inc) / n_steps,
                     hpmg_last_error());
      total_newton += its;
      stats[4 + step] += its;
      if (st == HPMG_OK) {
        // with no iteration from a lifted start the stored state is still the previous one
        state_at_u = its > 0 || extrapolated;
        HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, mg->nu0, 0.0, mg->nu0, mg->nup, s));
        have_prev = true;
        prev_inc = inc;
        done += inc;
        final_rel = rel;
        dt = std::min(1.0, 2.0 * inc);
        halvings = 0;
        continue;
      }
      if (st != HPMG_ERR_NOT_CONVERGED && st != HPMG_ERR_NONPOSITIVE_J && st != HPMG_ERR_NONFINITE &&
          st != HPMG_ERR_BREAKDOWN)
        return st;
      ++cuts;
      if (budget.exhausted || ++halvings > 6) {
        stats[0] = total_newton;
        stats[1] = total_lin;
        stats[2] = final_rel;
        stats[3] = cuts;
        if (budget.exhausted) {
          // u goes back to the last converged load level
          HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, mg->nu0, 0.0, mg->nu0, u, s));
          return fail(HPMG_ERR_NOT_CONVERGED, "newton_solve: total iteration budget spent (" +
                                                  std::to_string(total_newton) + " Newton, " +
                                                  std::to_string(total_lin) + " FCG iterations)");
        }
        return fail(HPMG_ERR_NOT_CONVERGED, "newton_solve: load increment failed after 6 halvings in a row");
      }
      HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, mg->nu0, 0.0, mg->nu0, u, s));
      state_at_u = false;
      dt = 0.5 * inc;
    }
  }
  stats[0] = total_newton;
  stats[1] = total_lin;
  stats[2] = final_rel;
  stats[3] = cuts;
  return HPMG_OK;
}

// ------------------------------------------------------------------------------------
// L-BFGS with the V-cycle as initial inverse Hessian (Section III-A).
// ------------------------------------------------------------------------------------
void hpmg_lbfgs_default_params(hpmg_lbfgs_params *p) {
  if (!p) return;
  p->rtol = 1e-8;
  p->max_its = 200;
  p->memory = 5;
  p->line_search = 1;
  p->monitor = 0;
}

static size_t lbfgs_bytes(int64_t n, int memory) {
  const size_t v = ((size_t)n * sizeof(double) + 255) / 256 * 256;
  return v * (size_t)(2 * memory + 4);
}

int hpmg_lbfgs_workspace_bytes(hpmg_mg mg, int memory, size_t *bytes) {
  int st = mg_check(mg, "lbfgs_workspace_bytes");
  if (st) return st;
  if (!bytes) return fail(HPMG_ERR_ARG, "lbfgs_workspace_bytes: null output");
  if (memory < 1 || memory > 32) return fail(HPMG_ERR_ARG, "lbfgs_workspace_bytes: 1 <= memory <= 32");
  *bytes = lbfgs_bytes(mg->lv[0].n, memory);
  return HPMG_OK;
}

int hpmg_lbfgs_solve(hpmg_op fine, hpmg_mg mg, double *u, const double *lift, const double *f_ext, int n_steps,
                     const hpmg_lbfgs_params *prm, const double *const *seeds, void *workspace,
                     size_t workspace_bytes, double *stats, void *stream) {
  // parameters first: nothing behind the handles is touched before they pass
  if (!u || !lift || !prm || !seeds || !stats || !workspace) return fail(HPMG_ERR_ARG, "lbfgs_solve: null argument");
  if (n_steps < 1 || n_steps > 60) return fail(HPMG_ERR_ARG, "lbfgs_solve: 1 <= n_steps <= 60");
  const int m = prm->memory;
  if (m < 1 || m > 32) return fail(HPMG_ERR_ARG, "lbfgs_solve: 1 <= memory <= 32");
  if (!(prm->rtol > 0.0) || prm->max_its < 1) return fail(HPMG_ERR_ARG, "lbfgs_solve: rtol > 0, max_its >= 1");
  int st = mg_check(mg, "lbfgs_solve");
  if (st) return st;
  if (!fine || fine != mg->lv[0].op) return fail(HPMG_ERR_ARG, "lbfgs_solve: operator is not the mg fine level");
  if (!fine->geo_ready) return fail(HPMG_ERR_ARG, "lbfgs_solve: call qdata_setup first");
  const int64_t n = mg->lv[0].n;
  if (workspace_bytes < lbfgs_bytes(n, m)) return fail(HPMG_ERR_WORKSPACE, "lbfgs_solve: workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(HPMG_ERR_WORKSPACE, "lbfgs_solve: workspace not 256-byte aligned");
  hipStream_t s = S(stream);
  const size_t vb = ((size_t)n * sizeof(double) + 255) / 256 * 256;
  char *w = static_cast<char *>(workspace);
  std::vector<double *> Sv(m), Yv(m);
  for (int i = 0; i < m; ++i) {
    Sv[i] = reinterpret_cast<double *>(w + (size_t)i * vb);
    Yv[i] = reinterpret_cast<double *>(w + (size_t)(m + i) * vb);
  }
  double *g = reinterpret_cast<double *>(w + (size_t)(2 * m) * vb);
  double *q = reinterpret_cast<double *>(w + (size_t)(2 * m + 1) * vb);
  double *gt = reinterpret_cast<double *>(w + (size_t)(2 * m + 2) * vb);
  double *ut = reinterpret_cast<double *>(w + (size_t)(2 * m + 3) * vb);
  double *d = q;  // the direction overwrites the two-loop vector in place
  auto dot = [&](const double *a, const double *b, double *out) -> int {
    HPMG_HIP(launch_dot(HPMG_F64, n, a, b, mg->red, mg->scal, s));
    int e = read_scalars(mg, 1, s);
    if (e) return e;
    *out = mg->host[0];
    return HPMG_OK;
  };
  double load = 0.0;  // fraction of the external load in the current step
  auto gradient = [&](const double *x, double *out, bool store, double *norm, unsigned *flags) -> int {
    HPMG_HIP(launch_residual(*fine, x, out, store, s));
    if (f_ext) HPMG_HIP(launch_axpby(HPMG_F64, n, -load, f_ext, 1.0, out, s));
    if (store) {
      fine->state_version++;
      fine->state_ready = true;
      fine->state32_ready = false;
    }
    int e = dot(out, out, norm);
    if (e) return e;
    *norm = std::sqrt(*norm);
    return hpmg_op_query_flags(fine, stream, flags);
  };
  for (int k = 0; k < 4 + n_steps; ++k) stats[k] = 0.0;
  const int64_t v0 = mg->n_vcycles;
  int total = 0, restarts = 0;
  double final_rel = 0.0;
  std::vector<double> rho(m), alph(m);
  for (int step = 0; step < n_steps; ++step) {
    load = (double)(step + 1) / n_steps;
    HPMG_HIP(launch_axpby(HPMG_F64, n, 1.0 / n_steps, lift, 1.0, u, s));
    // The V-cycle is built once per load step, on the tangent at the lifted start.
    double gn = 0.0;
    unsigned fl = 0;
    if ((st = gradient(u, g, true, &gn, &fl))) return st;
    if ((fl & (HPMG_FLAG_NONPOSITIVE_J | HPMG_FLAG_NONFINITE)) || !std::isfinite(gn))
      return fail(HPMG_ERR_NONPOSITIVE_J, "lbfgs_solve: inverted element at the start of a load step");
    if (has_redisc(mg) && (st = set_state(mg, u, s))) return st;
    if ((st = do_setup(mg, seeds, s))) return st;
    const double g0n = gn;
    int count = 0, head = 0, its = 0;  // pairs stored, slot of the next pair
    while (g0n > 0.0 && !(gn <= prm->rtol * g0n)) {
      if (its >= prm->max_its) {
        stats[0] = total + its;
        stats[1] = (double)(mg->n_vcycles - v0);
        stats[2] = gn / g0n;
        stats[3] = restarts;
        return fail(HPMG_ERR_NOT_CONVERGED, "lbfgs_solve: iteration limit");
      }
      // Two-loop recursion, newest pair first; then H0 = V-cycle; then oldest first.
      HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, g, 0.0, g, q, s));
      for (int j = 0; j < count; ++j) {
        const int i = (head - 1 - j + m) % m;
        double sq = 0.0;
        if ((st = dot(Sv[i], q, &sq))) return st;
        alph[i] = rho[i] * sq;
        HPMG_HIP(launch_axpby(HPMG_F64, n, -alph[i], Yv[i], 1.0, q, s));
      }
      if ((st = vcycle(mg, q, gt, s))) return st;  // r = H0 q, held in gt for now
      for (int j = count - 1; j >= 0; --j) {
        const int i = (head - 1 - j + m) % m;
        double yr = 0.0;
        if ((st = dot(Yv[i], gt, &yr))) return st;
        HPMG_HIP(launch_axpby(HPMG_F64, n, alph[i] - rho[i] * yr, Sv[i], 1.0, gt, s));
      }
      HPMG_HIP(launch_waxpby(HPMG_F64, n, -1.0, gt, 0.0, gt, d, s));
      double gd = 0.0;
      if ((st = dot(g, d, &gd))) return st;
      if (!(gd < 0.0)) {  // not a descent direction: forget the pairs, use H0 alone
        ++restarts;
        count = head = 0;
        if ((st = vcycle(mg, g, gt, s))) return st;
        HPMG_HIP(launch_waxpby(HPMG_F64, n, -1.0, gt, 0.0, gt, d, s));
        if ((st = dot(g, d, &gd))) return st;
        if (!(gd < 0.0)) return fail(HPMG_ERR_BREAKDOWN, "lbfgs_solve: V-cycle gives no descent direction");
      }
      double alpha = 1.0;
      if (prm->line_search) {
        // Critical-point step: secant root of g(a) = F(u + a d)^T d between 0 and 1.
        HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, u, 1.0, d, ut, s));
        double tn = 0.0;
        unsigned tf = 0;
        if ((st = gradient(ut, gt, false, &tn, &tf))) return st;
        double g1 = 0.0;
        if ((st = dot(gt, d, &g1))) return st;
        if (std::isfinite(g1) && !tf && g1 - gd > 0.0) alpha = std::min(1.5, std::max(0.1, gd / (gd - g1)));
        else if (!std::isfinite(g1) || tf) alpha = 0.5;
      }
      // Accept u + alpha d, halving alpha while the point is inadmissible.
      bool ok = false;
      double tn = 0.0;
      for (int bt = 0; bt < 7; ++bt) {
        HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, u, alpha, d, ut, s));
        unsigned tf = 0;
        if ((st = gradient(ut, gt, false, &tn, &tf))) return st;
        ok = std::isfinite(tn) && !(tf & (HPMG_FLAG_NONPOSITIVE_J | HPMG_FLAG_NONFINITE));
        if (ok) break;
        alpha *= 0.5;
      }
      if (!ok) return fail(HPMG_ERR_NONPOSITIVE_J, "lbfgs_solve: no admissible step length");
      // New pair s = alpha d, y = F(u_new) - F(u), kept when y^T s > 0.
      HPMG_HIP(launch_waxpby(HPMG_F64, n, alpha, d, 0.0, d, Sv[head], s));
      HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, gt, -1.0, g, Yv[head], s));
      double ys = 0.0;
      if ((st = dot(Yv[head], Sv[head], &ys))) return st;
      if (ys > 0.0) {
        rho[head] = 1.0 / ys;
        head = (head + 1) % m;
        count = std::min(count + 1, m);
      }
      HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, ut, 0.0, ut, u, s));
      HPMG_HIP(launch_waxpby(HPMG_F64, n, 1.0, gt, 0.0, gt, g, s));
      gn = tn;
      ++its;
      if (prm->monitor)
        std::fprintf(stderr, "[lbfgs] step %d it %d rel %.3e alpha %.3f pairs %d\n", step, its, gn / g0n, alpha,
                     count);
    }
    total += its;
    stats[4 + step] = its;
    final_rel = g0n > 0.0 ? gn / g0n : 0.0;
  }
  stats[0] = total;
  stats[1] = (double)(mg->n_vcycles - v0);
  stats[2] = final_rel;
  stats[3] = restarts;
  return HPMG_OK;
}

}  // extern "C"
