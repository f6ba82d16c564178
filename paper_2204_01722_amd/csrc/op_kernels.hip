// Fused element kernels of the matrix-free Neo-Hookean operator for gfx950.
//
// One workgroup processes one tile of ET consecutive elements with one thread per
// quadrature point (Q^3 per element).  Inside a kernel the element vector and the
// quadrature vector never leave the chip (Fig. libceedapi caption: E, B and D fused):
//
//   gather (E)  ->  sum-factorised interpolation, three 1D contractions staged in LDS
//   ->  collocated derivative B_xi B_I^+ (three more contractions, Section II-B)
//   ->  pointwise constitutive map in registers (Section II-A)
//   ->  transposed derivative and interpolation in LDS  ->  element records, summed per
//       node in a fixed order by a node-centric assembly pass (E^T, no atomics).
//
// Quadrature-point data are read/written as [tile][field][ET*Q^3] so each field of a
// tile is one contiguous, coalesced sweep.  Dirichlet flags ride in the top bits of the
// element-to-node map, so masking costs no extra memory traffic.
#include <cmath>
#include <cstdlib>
#include <string>
#include <type_traits>

#include "common.h"

namespace hpmg {
namespace {

template <int Q>
struct QT {
  static constexpr int Q3 = Q * Q * Q;
  static constexpr int ET = elems_per_tile(Q);
  static constexpr int NQ = ET * Q3;
  static constexpr int NT = tile_threads(Q);
};

// One 1D contraction along direction DIR of an array with dims (N1, N2, N3), N1
// fastest, for NC components stored back to back.  Output dims replace N_DIR by NO.
// TR = false: out_o = sum_i M[o][i] in_i (M is [NO][NI]);
// TR = true:  out_o = sum_i M[i][o] in_i (M is [NI][NO], the transpose is applied).
template <typename T, int N1, int N2, int N3, int DIR, int NO, bool TR, int NC>
__device__ __forceinline__ void stage(const T *__restrict__ in, T *__restrict__ out,
                                      const T *__restrict__ M, int q, bool live) {
  constexpr int NI = DIR == 0 ? N1 : DIR == 1 ? N2 : N3;
  constexpr int O1 = DIR == 0 ? NO : N1, O2 = DIR == 1 ? NO : N2, O3 = DIR == 2 ? NO : N3;
  constexpr int NIN = N1 * N2 * N3, NOUT = O1 * O2 * O3;
  constexpr int STR = DIR == 0 ? 1 : DIR == 1 ? N1 : N1 * N2;
  if (live && q < NOUT) {
    const int o1 = q % O1, o2 = (q / O1) % O2, o3 = q / (O1 * O2);
    const int o = DIR == 0 ? o1 : DIR == 1 ? o2 : o3;
    const int base = (DIR == 0 ? 0 : o1) + N1 * ((DIR == 1 ? 0 : o2) + N2 * (DIR == 2 ? 0 : o3));
    T m[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) m[i] = TR ? M[i * NO + o] : M[o * NI + i];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T acc = 0;
#pragma unroll
      for (int i = 0; i < NI; ++i) acc += m[i] * in[c * NIN + base + i * STR];
      out[c * NOUT + q] = acc;
    }
  }
}

// Nodes [NC][P^3] in `a` -> quadrature values [NC][Q^3] in `b` (a is overwritten).
template <typename T, int P, int Q, int NC>
__device__ __forceinline__ void interp(T *a, T *b, const T *sB, int q, bool live) {
  stage<T, P, P, P, 0, Q, false, NC>(a, b, sB, q, live);
  __syncthreads();
  stage<T, Q, P, P, 1, Q, false, NC>(b, a, sB, q, live);
  __syncthreads();
  stage<T, Q, Q, P, 2, Q, false, NC>(a, b, sB, q, live);
  __syncthreads();
}

// Quadrature values [NC][Q^3] in `b` -> nodes [NC][P^3] in `a` (transpose of interp).
template <typename T, int P, int Q, int NC>
__device__ __forceinline__ void interp_t(T *b, T *a, const T *sB, int q, bool live) {
  stage<T, Q, Q, Q, 2, P, true, NC>(b, a, sB, q, live);
  __syncthreads();
  stage<T, Q, Q, P, 1, P, true, NC>(a, b, sB, q, live);
  __syncthreads();
  stage<T, Q, P, P, 0, P, true, NC>(b, a, sB, q, live);
  __syncthreads();
}

// Reference gradient at quadrature point q from quadrature values (collocated
// derivative): G[c][k] = d(component c)/d xi_k.
//
// The empty asm statements pin each component's sums before the next component's LDS
// reads are issued.  Without them the scheduler hoists all 3 x 15 reads ahead of the
// first FMA, which costs ~50 extra VGPRs in FP64 and one wave per SIMD of occupancy.
template <typename T, int Q, int NC>
__device__ __forceinline__ void grad_q(const T *in, const T *sD, int q, T (&G)[NC][3]) {
  constexpr int Q3 = Q * Q * Q;
  const int q1 = q % Q, q2 = (q / Q) % Q, q3 = q / (Q * Q);
  T d1[Q], d2[Q], d3[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    d1[j] = sD[q1 * Q + j];
    d2[j] = sD[q2 * Q + j];
    d3[j] = sD[q3 * Q + j];
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    T g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      g0 += d1[j] * in[c * Q3 + j + Q * (q2 + Q * q3)];
      g1 += d2[j] * in[c * Q3 + q1 + Q * (j + Q * q3)];
      g2 += d3[j] * in[c * Q3 + q1 + Q * (q2 + Q * j)];
    }
    asm volatile("" : "+v"(g0), "+v"(g1), "+v"(g2)::"memory");
    G[c][0] = g0;
    G[c][1] = g1;
    G[c][2] = g2;
  }
}

// Transposed collocated derivative summed over directions: out[c][q] =
// sum_k sum_j D[j][q_k] f[c][k][.. j ..], f laid out [3][3][Q^3].
template <typename T, int Q>
__device__ __forceinline__ void grad_t_q(const T *f, const T *sD, int q, T *out, bool live) {
  constexpr int Q3 = Q * Q * Q;
  if (!live || q >= Q3) return;
  const int q1 = q % Q, q2 = (q / Q) % Q, q3 = q / (Q * Q);
  T d1[Q], d2[Q], d3[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    d1[j] = sD[j * Q + q1];
    d2[j] = sD[j * Q + q2];
    d3[j] = sD[j * Q + q3];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T acc = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      acc += d1[j] * f[(c * 3 + 0) * Q3 + j + Q * (q2 + Q * q3)];
      acc += d2[j] * f[(c * 3 + 1) * Q3 + q1 + Q * (j + Q * q3)];
      acc += d3[j] * f[(c * 3 + 2) * Q3 + q1 + Q * (q2 + Q * j)];
    }
    asm volatile("" : "+v"(acc)::"memory");
    out[c * Q3 + q] = acc;
  }
}

template <typename T>
__device__ __forceinline__ T det3(const T (&m)[3][3]) {
  return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
         m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
         m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

// adj(m) / det  (inverse), given det.
template <typename T>
__device__ __forceinline__ void inv3(const T (&m)[3][3], T det, T (&r)[3][3]) {
  const T id = T(1) / det;
  r[0][0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) * id;
  r[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) * id;
  r[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) * id;
  r[1][0] = (m[1][2] * m[2][0] - m[1][0] * m[2][2]) * id;
  r[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) * id;
  r[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) * id;
  r[2][0] = (m[1][0] * m[2][1] - m[1][1] * m[2][0]) * id;
  r[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) * id;
  r[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) * id;
}

// Symmetric tau stored as (xx, yy, zz, yz, xz, xy).
__device__ __forceinline__ constexpr int sym_index(int i, int j) {
  return i == j ? i : (i + j == 1 ? 5 : (i + j == 2 ? 4 : 3));
}

// Kinematics and Kirchhoff stress from the reference gradient G = du/dxi and the
// inverse geometric Jacobian D = dxi/dX (Section II-A):
//   H = G D, J - 1 = tr H + ((tr H)^2 - tr H^2)/2 + det H (no cancellation),
//   log J = log1p(J - 1), tau = mu (H + H^T + H H^T) + lambda log J I,
//   A = dxi/dx = D F^{-1}.
// J - 1 and log J are always evaluated in double.
template <typename T>
struct Kin {
  T A[3][3];
  T tau[6];
  T c;       // lambda log J
  double logJ;
  double Jm1;
  T H[3][3];
};

template <typename T>
__device__ __forceinline__ void kinematics(const T (&G)[3][3], const T (&D)[3][3], T mu, T lam,
                                           Kin<T> &k) {
  for (int i = 0; i < 3; ++i)
    for (int J = 0; J < 3; ++J) k.H[i][J] = G[i][0] * D[0][J] + G[i][1] * D[1][J] + G[i][2] * D[2][J];
  double Hd[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Hd[i][j] = (double)k.H[i][j];
  const double tr = Hd[0][0] + Hd[1][1] + Hd[2][2];
  double tr2 = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) tr2 += Hd[i][j] * Hd[j][i];
  k.Jm1 = tr + 0.5 * (tr * tr - tr2) + det3(Hd);
  k.logJ = log1p(k.Jm1);
  k.c = lam * (T)k.logJ;
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      T b = k.H[i][0] * k.H[j][0] + k.H[i][1] * k.H[j][1] + k.H[i][2] * k.H[j][2];
      T t = mu * (k.H[i][j] + k.H[j][i] + b);
      if (i == j) t += k.c;
      k.tau[sym_index(i, j)] = t;
    }
  T F[3][3], Fi[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) F[i][j] = (i == j ? T(1) : T(0)) + k.H[i][j];
  inv3(F, (T)(1.0 + k.Jm1), Fi);
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 3; ++j) k.A[a][j] = D[a][0] * Fi[0][j] + D[a][1] * Fi[1][j] + D[a][2] * Fi[2][j];
}

// Residual pointwise map: f[i][k] = W sum_j tau_ij A_kj  (W tau (dxi/dx)^T).
template <typename T>
__device__ __forceinline__ void residual_qf(const Kin<T> &k, T W, T (&f)[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) {
      T s = 0;
      for (int j = 0; j < 3; ++j) s += k.tau[sym_index(i, j)] * k.A[a][j];
      f[i][a] = W * s;
    }
}

// Jacobian pointwise map (eqs. Jacobian, dtau, depsilon in current configuration):
//   g = G A = grad_x du;  s = g tau + lambda tr(g) I + (mu - lambda log J)(g + g^T);
//   f = W s A^T.
template <typename T>
__device__ __forceinline__ void jacobian_qf(const T (&G)[3][3], const T (&A)[3][3], const T (&tau)[6],
                                            T c, T W, T mu, T lam, T (&f)[3][3]) {
  T g[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) g[i][j] = G[i][0] * A[0][j] + G[i][1] * A[1][j] + G[i][2] * A[2][j];
  const T trg = g[0][0] + g[1][1] + g[2][2];
  const T m2 = mu - c;
  T s[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T v = g[i][0] * tau[sym_index(0, j)] + g[i][1] * tau[sym_index(1, j)] + g[i][2] * tau[sym_index(2, j)];
      v += m2 * (g[i][j] + g[j][i]);
      if (i == j) v += lam * trg;
      s[i][j] = v;
    }
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) f[i][a] = W * (s[i][0] * A[a][0] + s[i][1] * A[a][1] + s[i][2] * A[a][2]);
}

// Adjoint pointwise map, written as the transpose of jacobian_qf: for a cotangent
// C = dw/dxi, s*(M) = M tau^T + lambda tr(M) I + (mu - c)(M + M^T) with M = C A, and
// f = W s*(M) A^T.
template <typename T>
__device__ __forceinline__ void adjoint_qf(const T (&C)[3][3], const T (&A)[3][3], const T (&tau)[6],
                                           T c, T W, T mu, T lam, T (&f)[3][3], T (&M)[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[i][j] = C[i][0] * A[0][j] + C[i][1] * A[1][j] + C[i][2] * A[2][j];
  const T trM = M[0][0] + M[1][1] + M[2][2];
  const T m2 = mu - c;
  T s[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      // (M tau^T)_ij = sum_m M_im tau_jm
      T v = M[i][0] * tau[sym_index(j, 0)] + M[i][1] * tau[sym_index(j, 1)] + M[i][2] * tau[sym_index(j, 2)];
      v += m2 * (M[i][j] + M[j][i]);
      if (i == j) v += lam * trM;
      s[i][j] = v;
    }
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) f[i][a] = W * (s[i][0] * A[a][0] + s[i][1] * A[a][1] + s[i][2] * A[a][2]);
}

// Jacobian pointwise map in the initial configuration (the S(E) form of the same
// model, Section V / Table different-storage): with dF = G D = grad_X du,
//   S  = mu I + (c - mu) C^-1                     (c = lambda log J),
//   dC = dF^T F + F^T dF,
//   dS = (mu - c) C^-1 dC C^-1 + (lambda / 2) tr(C^-1 dC) C^-1,
//   dP = dF S + F dS,   f = W dP D^T.
// hv holds grad_X u (9, row-major) and, when TUNED, C^-1 (6, symmetric) and c; the
// "native" form recomputes C^-1 and c from grad_X u (J - 1 without cancellation).
template <bool TUNED>
__device__ __forceinline__ void jacobian_qf_initial(const double (&G)[3][3], const double (&gv)[NGEO],
                                                    const double *hv, double mu, double lam,
                                                    double (&f)[3][3]) {
  double D[3][3], H[3][3], dF[3][3], F[3][3], Ci[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      D[k][J] = gv[1 + k * 3 + J];
      H[k][J] = hv[k * 3 + J];
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      dF[i][J] = G[i][0] * D[0][J] + G[i][1] * D[1][J] + G[i][2] * D[2][J];
      F[i][J] = (i == J ? 1.0 : 0.0) + H[i][J];
    }
  double c;
  if (TUNED) {
#pragma unroll
    for (int I = 0; I < 3; ++I)
#pragma unroll
      for (int J = 0; J < 3; ++J) Ci[I][J] = hv[9 + sym_index(I, J)];
    c = hv[15];
  } else {
    const double tr = H[0][0] + H[1][1] + H[2][2];
    double tr2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) tr2 += H[i][j] * H[j][i];
    const double Jm1 = tr + 0.5 * (tr * tr - tr2) + det3(H);
    c = lam * log1p(Jm1);
    double Fi[3][3];
    inv3(F, 1.0 + Jm1, Fi);
#pragma unroll
    for (int I = 0; I < 3; ++I)
#pragma unroll
      for (int J = 0; J < 3; ++J) Ci[I][J] = Fi[I][0] * Fi[J][0] + Fi[I][1] * Fi[J][1] + Fi[I][2] * Fi[J][2];
  }
  double dC[3][3];
#pragma unroll
  for (int I = 0; I < 3; ++I)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      double v = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) v += dF[a][I] * F[a][J] + F[a][I] * dF[a][J];
      dC[I][J] = v;
    }
  double M[3][3], tr = 0.0;
#pragma unroll
  for (int I = 0; I < 3; ++I)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      M[I][J] = Ci[I][0] * dC[0][J] + Ci[I][1] * dC[1][J] + Ci[I][2] * dC[2][J];
      if (I == J) tr += M[I][J];
    }
  double dS[3][3], Sm[3][3];
#pragma unroll
  for (int I = 0; I < 3; ++I)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      const double e1 = M[I][0] * Ci[0][J] + M[I][1] * Ci[1][J] + M[I][2] * Ci[2][J];
      dS[I][J] = (mu - c) * e1 + 0.5 * lam * tr * Ci[I][J];
      Sm[I][J] = (I == J ? mu : 0.0) + (c - mu) * Ci[I][J];
    }
  double dP[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      double v = 0.0;
#pragma unroll
      for (int K = 0; K < 3; ++K) v += dF[i][K] * Sm[K][J] + F[i][K] * dS[K][J];
      dP[i][J] = v;
    }
  const double W = gv[0];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) f[i][k] = W * (dP[i][0] * D[k][0] + dP[i][1] * D[k][1] + dP[i][2] * D[k][2]);
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.  Give
// every XCD a contiguous range of tiles so neighbouring elements (which share nodes,
// hence gathered values and atomic targets) run under the same L2.
__device__ __forceinline__ int64_t xcd_tile() {
  constexpr unsigned NX = 8;
  const unsigned b = blockIdx.x, G = gridDim.x;
  const unsigned m = G / NX, r = G % NX, x = b % NX, j = b / NX;
  return (int64_t)x * m + (x < r ? x : r) + j;
}

// Record traffic of FP64 operators of order 4 and 2 (P = 5, 3) goes through contiguous
// sweeps: the Jacobian kernel writes each tile's records from LDS as one run, and the
// assembly writes its output from LDS in whole-line nontemporal sweeps.  Records of up
// to 160 MiB (keep_records) are stored with plain stores, so that they stay in the
// 256 MB last-level cache for the assembly that follows; larger ones stream out with
// nontemporal stores.  Measured per apply, plain against nontemporal record stores:
// Q2 on 43^3 elements (52 MB of records) 87.2 against 92.5 us, Q4 on 34^3 (118 MB) 188
// against 201 us, Q2 on 60^3 (140 MB) 220 against 235 us; Q4 on 40^3 (192 MB) 354
// against 331 us, Q4 on 46^3 (292 MB) 549 against 515 us, Q2 on 86^3 (412 MB) 766
// against 724 us, Q4 on 68^3 (943 MB) 1750 against 1643 us; per-node stores: Q4 34^3
// 217 us, Q2 43^3 88.4 us, Q2 86^3 785 us.  In FP32 the per-node stores were as fast or
// faster.
template <typename T>
__host__ __device__ constexpr bool sweep_records(int P) {
  return std::is_same<T, double>::value && (P == 5 || P == 3);
}
template <typename T>
bool keep_records(int64_t E, int P) {
  return (double)E * P * P * P * 3 * sizeof(T) <= 160.0 * (1 << 20);
}

__device__ __forceinline__ double mat_mu(double mu0, const double *mu_e, int64_t e) {
  return mu_e ? mu_e[e] : mu0;
}

template <typename T>
__device__ __forceinline__ void load_tables(T *dst, const T *__restrict__ src, int off, int n, int t, int nt) {
  for (int i = t; i < n; i += nt) dst[i] = src[off + i];
}

// Loads the three components of a node (all issued before any is used) and writes them
// to LDS as [c][P^3]; constrained components become zero when `masked`.
template <typename S, typename T>
__device__ __forceinline__ void gather_node(const S *__restrict__ v, uint32_t w, bool masked, T *a, int q,
                                            int P3) {
  const S *p = v + (int64_t)(w & EMAP_ID_MASK) * 3;
  const S x0 = p[0], x1 = p[1], x2 = p[2];
  a[q] = (masked && ((w >> EMAP_BC_SHIFT) & 1u)) ? T(0) : (T)x0;
  a[P3 + q] = (masked && ((w >> (EMAP_BC_SHIFT + 1)) & 1u)) ? T(0) : (T)x1;
  a[2 * P3 + q] = (masked && ((w >> (EMAP_BC_SHIFT + 2)) & 1u)) ? T(0) : (T)x2;
}

// Writes the element's nodal result (LDS [c][P^3]) as records [e][a][c] for the
// node-centric assembly pass.
template <typename T>
__device__ __forceinline__ void store_record(T *__restrict__ ev, int64_t e, const T *a, int q, int P3) {
  T *p = ev + ((int64_t)e * P3 + q) * 3;
  const T x0 = a[q], x1 = a[P3 + q], x2 = a[2 * P3 + q];
  p[0] = x0;
  p[1] = x1;
  p[2] = x2;
}

// ------------------------------------------------------------------------------------
// a1: geometric factors.
// ------------------------------------------------------------------------------------
template <int P, int Q>
__global__ __launch_bounds__(QT<Q>::NT) void k_qdata(const uint32_t *__restrict__ emap,
                                                     const double *__restrict__ X,
                                                     const double *__restrict__ tab,
                                                     double *__restrict__ geo,
                                                     unsigned *__restrict__ flags, int64_t E) {
  using T = double;
  constexpr int Q3 = QT<Q>::Q3, ET = QT<Q>::ET, NQ = QT<Q>::NQ, NT = QT<Q>::NT, P3 = P * P * P;
  constexpr int S0 = 3 * Q3, S1 = 3 * Q3;
  __shared__ T sB[Q * P], sD[Q * Q], sW[Q];
  __shared__ T lds[ET * (S0 + S1)];
  const int tq = threadIdx.x, el = tq / Q3, q = tq % Q3;
  const int64_t tile = xcd_tile();
  const int64_t e = tile * ET + el;
  const bool live = tq < NQ && e < E;
  load_tables(sB, tab, TAB_B, Q * P, tq, NT);
  load_tables(sD, tab, TAB_D, Q * Q, tq, NT);
  load_tables(sW, tab, TAB_W, Q, tq, NT);
  T *a = lds + (live ? el : 0) * S0, *b = lds + ET * S0 + (live ? el : 0) * S1;
  if (live && q < P3) {
    const uint32_t node = emap[e * P3 + q] & EMAP_ID_MASK;
#pragma unroll
    for (int c = 0; c < 3; ++c) a[c * P3 + q] = X[(int64_t)node * 3 + c];
  }
  __syncthreads();
  interp<T, P, Q, 3>(a, b, sB, q, live);
  T G[3][3];
  if (live) grad_q<T, Q, 3>(b, sD, q, G);
  if (!live) return;
  const T det = det3(G);
  if (!(det > 0.0)) atomicOr(flags, det == det ? HPMG_FLAG_NONPOSITIVE_J : HPMG_FLAG_NONFINITE);
  T Di[3][3];
  inv3(G, det, Di);  // Di[k][J] = dxi_k / dX_J
  const int q1 = q % Q, q2 = (q / Q) % Q, q3 = q / (Q * Q);
  double *g = geo + tile * NGEO * NQ + tq;
  g[0] = sW[q1] * sW[q2] * sW[q3] * det;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int J = 0; J < 3; ++J) g[(1 + k * 3 + J) * NQ] = Di[k][J];
}

// ------------------------------------------------------------------------------------
// a4-a7: residual (FP64, MODE 4 below) and a5: Jacobian action from the stored
// linearisation (FP64 or FP32), with register-blocked 1D contractions.
//
// With one thread per point, each 1D contraction would cost a thread one LDS read per
// input of every output.  Here every contraction stage is run by "line tasks": a task
// owns one line of points along the contraction direction (for one component), reads
// the line once, forms all of its outputs in registers from the 1D table (the same for
// every lane, so it is read through the scalar cache, not LDS) and writes them back in
// place.  That is one LDS read and one write per point and stage.
// Nodal (P^3) and quadrature (Q^3) arrays share one Q^3 frame per component, indexed
// i1 + Q i2 + Q^2 i3, so the interpolation stages can work in place.  The pointwise
// work (state loads, quadrature function, gather, records) keeps the one-thread-per-
// point mapping and the tile layout of the other kernels.
// ------------------------------------------------------------------------------------

// First frame offset and stride of line r of a stage along DIR whose lines run over
// the other two directions with extents L1 (the faster one) and L2.
template <int Q, int DIR, int L1>
__device__ __forceinline__ int line_base(int r) {
  const int r1 = r % L1, r2 = r / L1;
  return DIR == 0 ? Q * (r1 + Q * r2) : DIR == 1 ? r1 + Q * Q * r2 : r1 + Q * r2;
}
template <int Q, int DIR>
__device__ __forceinline__ constexpr int line_step() {
  return DIR == 0 ? 1 : DIR == 1 ? Q : Q * Q;
}

// y = M x with M [NO][NI] row-major (TR = false) or y = M^T x with M [NI][NO] (TR = true).
template <typename T, int NI, int NO, bool TR>
__device__ __forceinline__ void line_apply(const T *__restrict__ M, const T (&x)[NI], T (&y)[NO]) {
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    T acc = 0;
#pragma unroll
    for (int i = 0; i < NI; ++i) acc += M[TR ? i * NO + o : o * NI + i] * x[i];
    y[o] = acc;
  }
}

// One in-place contraction stage along DIR (NI inputs -> NO outputs per line) of the
// three component frames of each of the tile's elements (element el at buf + el * ELS,
// component c at + c * Q^3).  Lines run over extents L1 x L2 of the other directions.
template <typename T, int Q, int DIR, int NI, int NO, bool TR, int L1, int L2, int ET, int ELS>
__device__ __forceinline__ void line_stage(T *buf, const T *__restrict__ M, int tid, int nt, int nel) {
  constexpr int NL = L1 * L2, TASKS = 3 * NL, Q3 = Q * Q * Q, ST = line_step<Q, DIR>();
  for (int t = tid; t < ET * TASKS; t += nt) {
    const int el = t / TASKS, r = t % TASKS, c = r / NL;
    if (el >= nel) break;
    T *p = buf + el * ELS + c * Q3 + line_base<Q, DIR, L1>(r % NL);
    T x[NI], y[NO];
#pragma unroll
    for (int i = 0; i < NI; ++i) x[i] = p[i * ST];
    line_apply<T, NI, NO, TR>(M, x, y);
#pragma unroll
    for (int i = 0; i < NO; ++i) p[i * ST] = y[i];
  }
}

template <typename T, int NI, int NO, bool TR, int ST>
__device__ __forceinline__ void line_task(T *p, const T *__restrict__ M) {
  T x[NI], y[NO];
#pragma unroll
  for (int i = 0; i < NI; ++i) x[i] = p[i * ST];
  line_apply<T, NI, NO, TR>(M, x, y);
#pragma unroll
  for (int i = 0; i < NO; ++i) p[i * ST] = y[i];
}

// MODE 0: the 16-scalar current-configuration state (sqrt(W) dxi/dx, tau, lambda log J;
// T = double or float).
// MODE 1 / 2: the initial-configuration forms, 19 / 26 scalars (geometry W, grad_X xi
// + grad_X u [+ C^-1, lambda log J]); T = double.
// MODE 3: the 20-scalar current-configuration form (dxi/dx, J, grad_X u, W): tau and
// lambda log J are rebuilt from grad_X u and J; T = double.
// MODE 4: the residual (du is u, unmasked; T = double): kinematics and the Kirchhoff
// flux from the geometry (W, dxi/dX), the 16-scalar state written to state_out when it
// is given, non-positive or non-finite J raised in flags.
// MODE 5: the Jacobian with the linearisation recomputed at u (T = double or float; u
// is converted to T): the kinematics of u from the geometry at every point, then the
// action on du as in MODE 0.
// SWEEP 1 / 2: the tile's element records leave LDS in contiguous sweeps (each store
// instruction covers whole cache lines) with plain (1) or nontemporal (2) stores, instead
// of three strided stores per node (0).  The two sweep kinds are separate instances: a
// run-time choice lets the compiler merge both stores into a plain one.
template <typename T, int P, int Q, int MODE, int SWEEP>
__global__ __launch_bounds__(QT<Q>::NT) void k_jacobian_lines(
    const uint32_t *__restrict__ emap, const T *__restrict__ du, const T *__restrict__ state,
    const double *__restrict__ geo, const double *__restrict__ sinit,
    const T *__restrict__ tab, double mu0, double lam0, const double *__restrict__ mu_e,
    const double *__restrict__ lam_e, T *__restrict__ ev, int64_t E, const double *__restrict__ stop,
    double *__restrict__ state_out, unsigned *__restrict__ flags, const double *__restrict__ u) {
  constexpr int NH = MODE == 2 ? 16 : MODE == 3 ? 19 : 9;
  static_assert(MODE != 4 || std::is_same<T, double>::value, "the residual form is FP64");
  if (stop && *stop != 0.0) return;  // a stopped PCG (uniform over the grid)
  constexpr int Q2 = Q * Q, Q3 = Q2 * Q, P3 = P * P * P, ET = QT<Q>::ET, NQ = QT<Q>::NQ, NT = QT<Q>::NT;
  // Per element: v [3][Q^3] (du, then its values at the points, then the z-derivative
  // G[c][2] and the z-flux in place, then the nodal result) and G [3][2][Q^3] (the x- and
  // y-derivatives, then the x- and y-flux): 9 Q^3 scalars, so that more tiles fit in LDS.
  constexpr int ELS = 9 * Q3;
  __shared__ T lds[ET * ELS];
  const int tq = threadIdx.x, el = tq / Q3, q = tq % Q3;
  const int64_t tile = xcd_tile();
  const int64_t e = tile * ET + el;
  const int nel = (int)((E - tile * ET) < ET ? (E - tile * ET) : ET);
  const bool live = tq < NQ && e < E;
  const T *tB = tab + TAB_B, *tD = tab + TAB_D;
  T *v = lds + (live ? el : 0) * ELS, *G = v + 3 * Q3;
  // Frame index of node q (q < P^3).
  const int qn = (q % P) + Q * ((q / P) % P) + Q2 * (q / (P * P));
  T sv[MODE == 0 ? NSTATE : 1];
  double gv[MODE == 0 ? 1 : MODE == 3 ? 1 : NGEO], hv[MODE == 0 ? 1 : NH];
  // FI: with P == Q every stage of 3 Q^2 line tasks per element decomposes a thread's
  // task alike (element, component, line), only the line's direction changes, and each
  // thread has at most one such task: its line offsets are formed once here (the same
  // arithmetic in the same order as the generic stages; measured 3-4 % faster for
  // order 4 in FP32 and order 2 in FP64, 1 % slower for order 4 in FP64, which keeps the
  // generic stages).
  constexpr bool FI = (P == Q) && (ET * 3 * Q2 <= NT) && !(std::is_same<T, double>::value && P == 5);
  const int e3 = tq / (3 * Q2), r3 = tq % (3 * Q2), c3 = r3 / Q2, ln3 = r3 % Q2;
  const bool a3 = tq < ET * 3 * Q2 && e3 < nel;
  T *const p3 = lds + (a3 ? e3 * ELS + c3 * Q3 : 0);
  const int lb0 = line_base<Q, 0, Q>(ln3), lb1 = line_base<Q, 1, Q>(ln3), lb2 = line_base<Q, 2, Q>(ln3);
  // MODE 5 runs the forward stages twice: on u first (pass 0), keeping the kinematics of
  // each point in registers, then, like every form, on du (pass 1).
  T kA[3][3], ktau[6], kc = T(0);
#pragma unroll 1
  for (int pass = MODE == 5 ? 0 : 1; pass < 2; ++pass) {
    if (live && q < P3) {
      const uint32_t w = emap[e * P3 + q];
      T x0, x1, x2;
      if (MODE == 5 && pass == 0) {
        const double *src = u + (int64_t)(w & EMAP_ID_MASK) * 3;
        x0 = (T)src[0], x1 = (T)src[1], x2 = (T)src[2];
      } else {
        const T *src = du + (int64_t)(w & EMAP_ID_MASK) * 3;
        x0 = src[0], x1 = src[1], x2 = src[2];
      }
      // u is taken whole (the residual, the recompute form's first pass); du has its
      // constrained components zeroed
      const uint32_t bc = (MODE == 4 || pass == 0) ? 0u : (w >> EMAP_BC_SHIFT);
      v[qn] = (bc & 1u) ? T(0) : x0;
      v[Q3 + qn] = ((bc >> 1) & 1u) ? T(0) : x1;
      v[2 * Q3 + qn] = ((bc >> 2) & 1u) ? T(0) : x2;
    }
    if (live && (MODE != 5 || pass == 0)) {
      if constexpr (MODE == 0) {
        const T *s = state + tile * NSTATE * NQ + tq;
#pragma unroll
        for (int f = 0; f < NSTATE; ++f) sv[f] = __builtin_nontemporal_load(s + f * NQ);
      } else if constexpr (MODE == 3) {
        gv[0] = __builtin_nontemporal_load(geo + tile * NGEO * NQ + tq);  // W only
        const double *h = sinit + tile * NINIT * NQ + tq;
#pragma unroll
        for (int f = 0; f < 9; ++f) hv[f] = __builtin_nontemporal_load(h + f * NQ);
#pragma unroll
        for (int f = 0; f < 10; ++f) hv[9 + f] = __builtin_nontemporal_load(h + (16 + f) * NQ);
      } else if constexpr (MODE == 4 || MODE == 5) {
        const double *g = geo + tile * NGEO * NQ + tq;
#pragma unroll
        for (int f = 0; f < NGEO; ++f) gv[f] = __builtin_nontemporal_load(g + f * NQ);
      } else {
        const double *g = geo + tile * NGEO * NQ + tq;
#pragma unroll
        for (int f = 0; f < NGEO; ++f) gv[f] = __builtin_nontemporal_load(g + f * NQ);
        const double *h = sinit + tile * NINIT * NQ + tq;
#pragma unroll
        for (int f = 0; f < NH; ++f) hv[f] = __builtin_nontemporal_load(h + f * NQ);
      }
    }
    __syncthreads();
    // Interpolation to the points, one direction at a time, in place.
    if constexpr (FI) {
      if (a3) line_task<T, P, Q, false, 1>(p3 + lb0, tB);
    } else {
      line_stage<T, Q, 0, P, Q, false, P, P, ET, ELS>(lds, tB, tq, NT, nel);
    }
    __syncthreads();
    if constexpr (FI) {
      if (a3) line_task<T, P, Q, false, Q>(p3 + lb1, tB);
    } else {
      line_stage<T, Q, 1, P, Q, false, Q, P, ET, ELS>(lds, tB, tq, NT, nel);
    }
    __syncthreads();
    if constexpr (FI) {
      if (a3) line_task<T, P, Q, false, Q2>(p3 + lb2, tB);
    } else {
      line_stage<T, Q, 2, P, Q, false, Q, Q, ET, ELS>(lds, tB, tq, NT, nel);
    }
    __syncthreads();
    // Collocated derivative in the three directions: G[c][k] = D_k v[c] for k = 0, 1 into
    // G, then (once every x and y line has read v) D_z v[c] in place over v[c].
    {
      constexpr int TASKS = 6 * Q2;
      for (int t = tq; t < ET * TASKS; t += NT) {
        const int te = t / TASKS, r = t % TASKS, ck = r / Q2, c = ck / 2, k = ck % 2, ln = r % Q2;
        if (te >= nel) break;
        const T *src = lds + te * ELS + c * Q3;
        T *dst = lds + te * ELS + (3 + ck) * Q3;
        T x[Q], y[Q];
        if (k == 0) {
          const int b0 = line_base<Q, 0, Q>(ln);
#pragma unroll
          for (int i = 0; i < Q; ++i) x[i] = src[b0 + i];
          line_apply<T, Q, Q, false>(tD, x, y);
#pragma unroll
          for (int i = 0; i < Q; ++i) dst[b0 + i] = y[i];
        } else {
          const int b1 = line_base<Q, 1, Q>(ln);
#pragma unroll
          for (int i = 0; i < Q; ++i) x[i] = src[b1 + i * Q];
          line_apply<T, Q, Q, false>(tD, x, y);
#pragma unroll
          for (int i = 0; i < Q; ++i) dst[b1 + i * Q] = y[i];
        }
      }
    }
    __syncthreads();
    if constexpr (FI) {
      if (a3) line_task<T, Q, Q, false, Q2>(p3 + lb2, tD);
    } else {
      constexpr int TASKS = 3 * Q2;
      for (int t = tq; t < ET * TASKS; t += NT) {
        const int te = t / TASKS, r = t % TASKS, c = r / Q2, ln = r % Q2;
        if (te >= nel) break;
        T *p = lds + te * ELS + c * Q3 + line_base<Q, 2, Q>(ln);
        T x[Q], y[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) x[i] = p[i * Q2];
        line_apply<T, Q, Q, false>(tD, x, y);
#pragma unroll
        for (int i = 0; i < Q; ++i) p[i * Q2] = y[i];
      }
    }
    __syncthreads();
    if constexpr (MODE == 5) {
      if (pass == 0) {
        // the kinematics of u at this point, kept for the du pass
        if (live) {
          T Gu[3][3], D[3][3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            Gu[c][0] = G[(c * 2) * Q3 + q];
            Gu[c][1] = G[(c * 2 + 1) * Q3 + q];
            Gu[c][2] = v[c * Q3 + q];
          }
#pragma unroll
          for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int J = 0; J < 3; ++J) D[k][J] = (T)gv[1 + k * 3 + J];
          Kin<T> k;
          kinematics(Gu, D, (T)mat_mu(mu0, mu_e, e), (T)mat_mu(lam0, lam_e, e), k);
#pragma unroll
          for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) kA[i][j] = k.A[i][j];
#pragma unroll
          for (int m = 0; m < 6; ++m) ktau[m] = k.tau[m];
          kc = k.c;
        }
        __syncthreads();  // every point has read its gradient before du overwrites the frames
      }
    }
  }  // pass
  // Quadrature function, one thread per point, flux written over the gradient
  // (components k = 0, 1 in G, k = 2 in v).
  if (live) {
    T Gq[3][3], f[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Gq[c][0] = G[(c * 2) * Q3 + q];
      Gq[c][1] = G[(c * 2 + 1) * Q3 + q];
      Gq[c][2] = v[c * Q3 + q];
    }
    if constexpr (MODE == 0) {
      T A[3][3], tau[6];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) A[k][j] = sv[k * 3 + j];
#pragma unroll
      for (int m = 0; m < 6; ++m) tau[m] = sv[9 + m];
      const T c = sv[15], W = T(1);  // the weight is in the scaled dxi/dx
      const T mu = (T)mat_mu(mu0, mu_e, e), lam = (T)mat_mu(lam0, lam_e, e);
      jacobian_qf(Gq, A, tau, c, W, mu, lam, f);
    } else if constexpr (MODE == 3) {
      const double mu = mat_mu(mu0, mu_e, e), lam = mat_mu(lam0, lam_e, e);
      double A[3][3], tau[6];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) A[k][j] = hv[9 + k * 3 + j];
      const double c = lam * log1p(hv[18]);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
          const double hh = hv[i * 3] * hv[j * 3] + hv[i * 3 + 1] * hv[j * 3 + 1] + hv[i * 3 + 2] * hv[j * 3 + 2];
          tau[sym_index(i, j)] = mu * (hv[i * 3 + j] + hv[j * 3 + i] + hh) + (i == j ? c : 0.0);
        }
      jacobian_qf(Gq, A, tau, c, gv[0], mu, lam, f);
    } else if constexpr (MODE == 5) {
      jacobian_qf(Gq, kA, ktau, kc, (T)gv[0], (T)mat_mu(mu0, mu_e, e), (T)mat_mu(lam0, lam_e, e), f);
    } else if constexpr (MODE == 4) {
      double D[3][3];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int J = 0; J < 3; ++J) D[k][J] = gv[1 + k * 3 + J];
      Kin<double> k;
      kinematics(Gq, D, mat_mu(mu0, mu_e, e), mat_mu(lam0, lam_e, e), k);
      if (!(k.Jm1 > -1.0)) atomicOr(flags, k.Jm1 == k.Jm1 ? HPMG_FLAG_NONPOSITIVE_J : HPMG_FLAG_NONFINITE);
      residual_qf(k, gv[0], f);
      if (state_out) {
        // sqrt(W) dxi/dx, tau, lambda log J (the weight rides in the scaled dxi/dx)
        double *so = state_out + tile * NSTATE * NQ + tq;
        const double sw = sqrt(gv[0]);
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
#pragma unroll
          for (int j = 0; j < 3; ++j) so[(kk * 3 + j) * NQ] = sw * k.A[kk][j];
#pragma unroll
        for (int m = 0; m < 6; ++m) so[(9 + m) * NQ] = k.tau[m];
        so[15 * NQ] = k.c;
      }
    } else {
      jacobian_qf_initial<MODE == 2>(Gq, gv, hv, mat_mu(mu0, mu_e, e), mat_mu(lam0, lam_e, e), f);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      G[(i * 2) * Q3 + q] = f[i][0];
      G[(i * 2 + 1) * Q3 + q] = f[i][1];
      v[i * Q3 + q] = f[i][2];
    }
  }
  __syncthreads();
  // Transposed derivative, x and y directions in place on the flux arrays.
  {
    constexpr int TASKS = 6 * Q2;
    for (int t = tq; t < ET * TASKS; t += NT) {
      const int te = t / TASKS, r = t % TASKS, ck = r / Q2, c = ck / 2, k = ck % 2, ln = r % Q2;
      if (te >= nel) break;
      T *p = lds + te * ELS + (3 + c * 2 + k) * Q3;
      T x[Q], y[Q];
      if (k == 0) {
        const int b0 = line_base<Q, 0, Q>(ln);
#pragma unroll
        for (int i = 0; i < Q; ++i) x[i] = p[b0 + i];
        line_apply<T, Q, Q, true>(tD, x, y);
#pragma unroll
        for (int i = 0; i < Q; ++i) p[b0 + i] = y[i];
      } else {
        const int b1 = line_base<Q, 1, Q>(ln);
#pragma unroll
        for (int i = 0; i < Q; ++i) x[i] = p[b1 + i * Q];
        line_apply<T, Q, Q, true>(tD, x, y);
#pragma unroll
        for (int i = 0; i < Q; ++i) p[b1 + i * Q] = y[i];
      }
    }
  }
  __syncthreads();
  // z direction: h = D_z^T f_z + (x and y parts), then the first transposed
  // interpolation stage (B_z^T, Q -> P) in registers; the result goes to v, over the
  // z-flux line it was formed from.
  if constexpr (FI) {
    if (a3) {
      const T *fxy = p3 + (3 + c3) * Q3 + lb2;
      T *o = p3 + lb2;
      T x[Q], y[Q], z[P];
#pragma unroll
      for (int i = 0; i < Q; ++i) x[i] = o[i * Q2];
      line_apply<T, Q, Q, true>(tD, x, y);
#pragma unroll
      for (int i = 0; i < Q; ++i) y[i] += fxy[i * Q2] + fxy[Q3 + i * Q2];
      line_apply<T, Q, P, true>(tB, y, z);
#pragma unroll
      for (int i = 0; i < P; ++i) o[i * Q2] = z[i];
    }
  } else {
    constexpr int TASKS = 3 * Q2;
    for (int t = tq; t < ET * TASKS; t += NT) {
      const int te = t / TASKS, r = t % TASKS, c = r / Q2, ln = r % Q2;
      if (te >= nel) break;
      const int b2 = line_base<Q, 2, Q>(ln);
      const T *fxy = lds + te * ELS + (3 + c * 2) * Q3 + b2;
      T *o = lds + te * ELS + c * Q3 + b2;
      T x[Q], y[Q], z[P];
#pragma unroll
      for (int i = 0; i < Q; ++i) x[i] = o[i * Q2];
      line_apply<T, Q, Q, true>(tD, x, y);
#pragma unroll
      for (int i = 0; i < Q; ++i) y[i] += fxy[i * Q2] + fxy[Q3 + i * Q2];
      line_apply<T, Q, P, true>(tB, y, z);
#pragma unroll
      for (int i = 0; i < P; ++i) o[i * Q2] = z[i];
    }
  }
  __syncthreads();
  if constexpr (FI) {
    if (a3) line_task<T, Q, P, true, Q>(p3 + lb1, tB);
  } else {
    line_stage<T, Q, 1, Q, P, true, Q, P, ET, ELS>(lds, tB, tq, NT, nel);
  }
  __syncthreads();
  if constexpr (FI) {
    if (a3) line_task<T, Q, P, true, 1>(p3 + lb0, tB);
  } else {
    line_stage<T, Q, 0, Q, P, true, P, P, ET, ELS>(lds, tB, tq, NT, nel);
  }
  __syncthreads();
  if constexpr (SWEEP > 0) {
    // records [e][a][c] of the tile's elements are one contiguous run of nel P^3 3 values
    T *o = ev + tile * (int64_t)(ET * P3 * 3);
    const int nd = nel * P3 * 3;
    for (int d = tq; d < nd; d += NT) {
      const int r = d / 3, c = d - 3 * r, te = r / P3, a = r - te * P3;
      const int an = (a % P) + Q * ((a / P) % P) + Q2 * (a / (P * P));
      if constexpr (SWEEP == 1)
        o[d] = lds[te * ELS + c * Q3 + an];
      else
        __builtin_nontemporal_store(lds[te * ELS + c * Q3 + an], o + d);
    }
  } else if (live && q < P3) {
    T *o = ev + ((int64_t)e * P3 + q) * 3;
    const T y0 = v[qn], y1 = v[Q3 + qn], y2 = v[2 * Q3 + qn];
    o[0] = y0;
    o[1] = y1;
    o[2] = y2;
  }
}

// Launches k_jacobian_lines with the record-store form for its order, precision and size.
template <typename T, int P, int Q, int MODE, typename... A>
void lines_launch(unsigned tiles, hipStream_t s, bool keep, A... a) {
  if constexpr (sweep_records<T>(P)) {
    if (keep)
      k_jacobian_lines<T, P, Q, MODE, 1><<<tiles, QT<Q>::NT, 0, s>>>(a...);
    else
      k_jacobian_lines<T, P, Q, MODE, 2><<<tiles, QT<Q>::NT, 0, s>>>(a...);
  } else {
    k_jacobian_lines<T, P, Q, MODE, 0><<<tiles, QT<Q>::NT, 0, s>>>(a...);
  }
}

// ------------------------------------------------------------------------------------
// Alternative linearisations at u, per point, [tile][26][ET*Q^3]: grad_X u (9),
// C^-1 (6), lambda log J (1), dxi/dx (9), J - 1 (1).  With the constant W and
// grad_X xi, fields 0-8 are the 19-scalar initial-configuration "native" form, 0-15 the
// 26-scalar "tuned" form; fields 0-8 and 16-25 with W are the 20-scalar current-
// configuration form (dxi/dx, J, grad_X u, W).
// ------------------------------------------------------------------------------------
template <int P, int Q>
__global__ __launch_bounds__(QT<Q>::NT) void k_state_initial(
    const uint32_t *__restrict__ emap, const double *__restrict__ u, const double *__restrict__ geo,
    const double *__restrict__ tab, double mu0, double lam0, const double *__restrict__ mu_e,
    const double *__restrict__ lam_e, double *__restrict__ sinit, unsigned *__restrict__ flags, int64_t E) {
  using T = double;
  constexpr int Q3 = QT<Q>::Q3, ET = QT<Q>::ET, NQ = QT<Q>::NQ, NT = QT<Q>::NT, P3 = P * P * P;
  constexpr int S0 = 3 * Q3;
  __shared__ T sB[Q * P], sD[Q * Q];
  __shared__ T lds[2 * ET * S0];
  const int tq = threadIdx.x, el = tq / Q3, q = tq % Q3;
  const int64_t tile = xcd_tile();
  const int64_t e = tile * ET + el;
  const bool live = tq < NQ && e < E;
  load_tables(sB, tab, TAB_B, Q * P, tq, NT);
  load_tables(sD, tab, TAB_D, Q * Q, tq, NT);
  T *a = lds + (live ? el : 0) * S0, *b = lds + ET * S0 + (live ? el : 0) * S0;
  if (live && q < P3) gather_node(u, emap[e * P3 + q], false, a, q, P3);
  __syncthreads();
  interp<T, P, Q, 3>(a, b, sB, q, live);
  if (!live) return;
  T G[3][3], D[3][3];
  grad_q<T, Q, 3>(b, sD, q, G);
  const double *g = geo + tile * NGEO * NQ + tq;
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int J = 0; J < 3; ++J) D[k][J] = g[(1 + k * 3 + J) * NQ];
  Kin<T> k;
  kinematics(G, D, mat_mu(mu0, mu_e, e), mat_mu(lam0, lam_e, e), k);
  if (!(k.Jm1 > -1.0)) atomicOr(flags, k.Jm1 == k.Jm1 ? HPMG_FLAG_NONPOSITIVE_J : HPMG_FLAG_NONFINITE);
  T F[3][3], Fi[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) F[i][j] = (i == j ? 1.0 : 0.0) + k.H[i][j];
  inv3(F, 1.0 + k.Jm1, Fi);
  double *o = sinit + tile * NINIT * NQ + tq;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int J = 0; J < 3; ++J) o[(i * 3 + J) * NQ] = k.H[i][J];
#pragma unroll
  for (int I = 0; I < 3; ++I)
#pragma unroll
    for (int J = I; J < 3; ++J)
      o[(9 + sym_index(I, J)) * NQ] = Fi[I][0] * Fi[J][0] + Fi[I][1] * Fi[J][1] + Fi[I][2] * Fi[J][2];
  o[15 * NQ] = k.c;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) o[(16 + a * 3 + j) * NQ] = k.A[a][j];
  o[25 * NQ] = k.Jm1;
}

// ------------------------------------------------------------------------------------
// External dead loads (eq. variational-form, right-hand side).
// Body force: per element int phi_a dV = sum_q B3[q][a] W_q, a transposed
// interpolation of the point weights, times rho0 g; element records.
// ------------------------------------------------------------------------------------
template <int P, int Q>
__global__ __launch_bounds__(QT<Q>::NT) void k_body_load(const double *__restrict__ geo,
                                                         const double *__restrict__ tab, double g0, double g1,
                                                         double g2, double *__restrict__ ev, int64_t E) {
  using T = double;
  constexpr int Q3 = QT<Q>::Q3, ET = QT<Q>::ET, NQ = QT<Q>::NQ, NT = QT<Q>::NT, P3 = P * P * P;
  __shared__ T sB[Q * P];
  __shared__ T lds[2 * ET * Q3];
  const int tq = threadIdx.x, el = tq / Q3, q = tq % Q3;
  const int64_t tile = xcd_tile();
  const int64_t e = tile * ET + el;
  const bool live = tq < NQ && e < E;
  load_tables(sB, tab, TAB_B, Q * P, tq, NT);
  T *a = lds + (live ? el : 0) * Q3, *b = lds + ET * Q3 + (live ? el : 0) * Q3;
  if (live) b[q] = geo[tile * NGEO * NQ + tq];  // W
  __syncthreads();
  interp_t<T, P, Q, 1>(b, a, sB, q, live);
  if (live && q < P3) {
    double *o = ev + ((int64_t)e * P3 + q) * 3;
    const T v = a[q];
    o[0] = v * g0;
    o[1] = v * g1;
    o[2] = v * g2;
  }
}

// Traction on element faces, one thread per face: the face's P^2 nodes (local face
// 0..5 = xi_1 = -1, +1, xi_2 = -1, +1, xi_3 = -1, +1), area element |X_,s x X_,r| from
// the in-face derivatives at the Q^2 Gauss points, records [face][P^2][3] = int phi t dA
// and the node of each record.
template <int P, int Q>
__global__ void k_traction_load(const double *__restrict__ X, const int32_t *__restrict__ elem_nodes,
                                const int32_t *__restrict__ face_elem, const int32_t *__restrict__ face_id,
                                const double *__restrict__ tab, double t0, double t1, double t2, int64_t nf,
                                int64_t E, double *__restrict__ rec, int32_t *__restrict__ rec_node,
                                unsigned *__restrict__ flags) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int32_t e = face_elem[f], id = face_id[f];
  double *out = rec + f * P * P * 3;
  int32_t *nodes = rec_node + f * P * P;
  if (e < 0 || e >= E || id < 0 || id > 5) {  // reported to the host, nothing written
    atomicOr(flags, 4u);
    for (int k = 0; k < P * P; ++k) {
      nodes[k] = -1;
      out[3 * k] = out[3 * k + 1] = out[3 * k + 2] = 0.0;
    }
    return;
  }
  const int d = id / 2, ad = (id % 2) ? P - 1 : 0;
  const int sd = d == 0 ? 1 : 0, rd = d == 2 ? 1 : 2;  // in-face directions, s < r
  const int str[3] = {1, P, P * P};
  double x[P * P][3];
  for (int c = 0; c < P; ++c)
    for (int b = 0; b < P; ++b) {
      const int a = ad * str[d] + b * str[sd] + c * str[rd];
      const int32_t n = elem_nodes[(int64_t)e * P * P * P + a];
      nodes[b + P * c] = n;
      for (int k = 0; k < 3; ++k) x[b + P * c][k] = X[(int64_t)n * 3 + k];
    }
  double acc[P * P];
  for (int k = 0; k < P * P; ++k) acc[k] = 0.0;
  const double *B = tab + TAB_B, *G = tab + TAB_G, *w = tab + TAB_W;
  for (int j = 0; j < Q; ++j)
    for (int i = 0; i < Q; ++i) {
      double ts[3] = {0, 0, 0}, tr[3] = {0, 0, 0};
      for (int c = 0; c < P; ++c)
        for (int b = 0; b < P; ++b) {
          const double gs = G[i * P + b] * B[j * P + c], gr = B[i * P + b] * G[j * P + c];
          for (int k = 0; k < 3; ++k) {
            ts[k] += gs * x[b + P * c][k];
            tr[k] += gr * x[b + P * c][k];
          }
        }
      const double n0 = ts[1] * tr[2] - ts[2] * tr[1], n1 = ts[2] * tr[0] - ts[0] * tr[2],
                   n2 = ts[0] * tr[1] - ts[1] * tr[0];
      const double dA = sqrt(n0 * n0 + n1 * n1 + n2 * n2) * w[i] * w[j];
      for (int c = 0; c < P; ++c)
        for (int b = 0; b < P; ++b) acc[b + P * c] += B[i * P + b] * B[j * P + c] * dA;
    }
  for (int k = 0; k < P * P; ++k) {
    out[3 * k] = acc[k] * t0;
    out[3 * k + 1] = acc[k] * t1;
    out[3 * k + 2] = acc[k] * t2;
  }
}

// ------------------------------------------------------------------------------------
// a8: diagonal.  Per quadrature point and component i, the 3x3 block
//   K^(i)_kl = W [ (A tau A^T)_kl + (mu - c)(A A^T)_kl + (lambda + mu - c) A_ki A_li ]
// (from the stored sqrt(W) A the weight comes out of the products itself)
// (the Jacobian map with G = e_i grad(phi)^T); the node value is
//   sum_q sum_kl K^(i)_kl dphi/dxi_k dphi/dxi_l,
// a tensor product of the 1D elementwise tables B*B, B*G, G*G, contracted in three
// transposed 1D stages for each of the six (k, l) pairs.
// ------------------------------------------------------------------------------------
template <typename T, int P, int Q>
__global__ __launch_bounds__(QT<Q>::NT) void k_diagonal(
    const uint32_t *__restrict__ emap, const T *__restrict__ state, const T *__restrict__ tab,
    double mu0, double lam0, const double *__restrict__ mu_e, const double *__restrict__ lam_e,
    T *__restrict__ ev, int64_t E) {
  constexpr int Q3 = QT<Q>::Q3, ET = QT<Q>::ET, NQ = QT<Q>::NQ, NT = QT<Q>::NT, P3 = P * P * P;
  constexpr int S0 = 3 * Q3, S1 = 3 * Q3;
  __shared__ T sBB[Q * P], sBG[Q * P], sGG[Q * P];
  __shared__ T lds[ET * (S0 + S1)];
  const int tq = threadIdx.x, el = tq / Q3, q = tq % Q3;
  const int64_t tile = xcd_tile();
  const int64_t e = tile * ET + el;
  const bool live = tq < NQ && e < E;
  load_tables(sBB, tab, TAB_BB, Q * P, tq, NT);
  load_tables(sBG, tab, TAB_BG, Q * P, tq, NT);
  load_tables(sGG, tab, TAB_GG, Q * P, tq, NT);
  T *a = lds + (live ? el : 0) * S0, *b = lds + ET * S0 + (live ? el : 0) * S1;
  T K[3][6];  // [component][pair]
  if (live) {
    T A[3][3], tau[6];
    const T *s = state + tile * NSTATE * NQ + tq;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int j = 0; j < 3; ++j) A[k][j] = s[(k * 3 + j) * NQ];
#pragma unroll
    for (int m = 0; m < 6; ++m) tau[m] = s[(9 + m) * NQ];
    const T c = s[15 * NQ], W = T(1);  // the weight is in the scaled dxi/dx
    const T mu = (T)mat_mu(mu0, mu_e, e), lam = (T)mat_mu(lam0, lam_e, e);
    T AT[3][3];  // (A tau)
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 3; ++j)
        AT[k][j] = A[k][0] * tau[sym_index(0, j)] + A[k][1] * tau[sym_index(1, j)] + A[k][2] * tau[sym_index(2, j)];
    const int pk[6] = {0, 1, 2, 1, 0, 0}, pl[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
    for (int p = 0; p < 6; ++p) {
      const int k = pk[p], l = pl[p];
      const T m1 = AT[k][0] * A[l][0] + AT[k][1] * A[l][1] + AT[k][2] * A[l][2];
      const T m2 = A[k][0] * A[l][0] + A[k][1] * A[l][1] + A[k][2] * A[l][2];
      const T sc = (k == l) ? W : T(2) * W;
#pragma unroll
      for (int i = 0; i < 3; ++i) K[i][p] = sc * (m1 + (mu - c) * m2 + (lam + mu - c) * A[k][i] * A[l][i]);
    }
  }
  T acc[3] = {0, 0, 0};
  const int pk[6] = {0, 1, 2, 1, 0, 0}, pl[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    if (live) {
#pragma unroll
      for (int i = 0; i < 3; ++i) b[i * Q3 + q] = K[i][p];
    }
    __syncthreads();
    const int k = pk[p], l = pl[p];
    const T *t1 = (k == 0 && l == 0) ? sGG : (k == 0 || l == 0) ? sBG : sBB;
    const T *t2 = (k == 1 && l == 1) ? sGG : (k == 1 || l == 1) ? sBG : sBB;
    const T *t3 = (k == 2 && l == 2) ? sGG : (k == 2 || l == 2) ? sBG : sBB;
    stage<T, Q, Q, Q, 2, P, true, 3>(b, a, t3, q, live);
    __syncthreads();
    stage<T, Q, Q, P, 1, P, true, 3>(a, b, t2, q, live);
    __syncthreads();
    stage<T, Q, P, P, 0, P, true, 3>(b, a, t1, q, live);
    __syncthreads();
    if (live && q < P3) {
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[i] += a[i * P3 + q];
    }
  }
  if (live && q < P3) {
    T *p = ev + ((int64_t)e * P3 + q) * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) p[c] = acc[c];
  }
}


// ------------------------------------------------------------------------------------
// Element matrices of an order-1 coarse operator on the fine quadrature (24 x 24 per
// element): column j = (node b, component k) is the element response to the unit
// nodal vector e_j, i.e. the Jacobian pointwise map applied to the rank-one gradient
// e_k (grad_xi phi_b)^T and integrated against every test function.  Exactly the
// matrix-free coarse operator, stored densely (3.7x fewer bytes per apply than the
// fine-quadrature linearisation at Q = 5).
// ------------------------------------------------------------------------------------
constexpr int ELB = 8;  // elements per workgroup (8 x 24 = 192 threads)
constexpr int ELMAT_PACKED = 300;  // 24 x 25 / 2 entries of the symmetric element matrix
__device__ __forceinline__ constexpr int elmat_index(int r, int j) { return r * (47 - r) / 2 + j; }

// T: precision of the state, tables, arithmetic and result (FP32 for the mixed-precision
// preconditioner, FP64 otherwise).
template <typename T, int Q>
__global__ __launch_bounds__(ELB * 24) void k_elmat_build(const T *__restrict__ state,
                                                          const T *__restrict__ tab, double mu0,
                                                          double lam0, const double *__restrict__ mu_e,
                                                          const double *__restrict__ lam_e,
                                                          T *__restrict__ K, int64_t E) {
  constexpr int Q3 = Q * Q * Q, ET = QT<Q>::ET, NQ = QT<Q>::NQ;
  __shared__ T sB[Q * 2], sG[Q * 2];
  const int t = threadIdx.x, el = t / 24, j = t % 24;
  const int64_t e = (int64_t)blockIdx.x * ELB + el;
  if (t < 2 * Q) {
    sB[t] = tab[TAB_B + t];
    sG[t] = tab[TAB_G + t];
  }
  __syncthreads();
  if (e >= E) return;
  const int b = j / 3, k = j % 3, b1 = b & 1, b2 = (b >> 1) & 1, b3 = b >> 2;
  const T mu = (T)mat_mu(mu0, mu_e, e), lam = (T)mat_mu(lam0, lam_e, e);
  const T *s = state + ((e / ET) * NSTATE) * NQ + (e % ET) * Q3;
  T acc[24];
#pragma unroll
  for (int r = 0; r < 24; ++r) acc[r] = T(0);
  for (int q = 0; q < Q3; ++q) {
    const int q1 = q % Q, q2 = (q / Q) % Q, q3 = q / (Q * Q);
    T A[3][3], tau[6];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) A[a][jj] = s[(a * 3 + jj) * NQ + q];
#pragma unroll
    for (int m = 0; m < 6; ++m) tau[m] = s[(9 + m) * NQ + q];
    const T c = s[15 * NQ + q], W = T(1);  // the weight is in the scaled dxi/dx
    // reference gradient of basis b at q
    const T Bx = sB[q1 * 2 + b1], By = sB[q2 * 2 + b2], Bz = sB[q3 * 2 + b3];
    const T Gx = sG[q1 * 2 + b1], Gy = sG[q2 * 2 + b2], Gz = sG[q3 * 2 + b3];
    const T dp[3] = {Gx * By * Bz, Bx * Gy * Bz, Bx * By * Gz};
    T v[3], w[3];
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) v[jj] = dp[0] * A[0][jj] + dp[1] * A[1][jj] + dp[2] * A[2][jj];
#pragma unroll
    for (int jj = 0; jj < 3; ++jj)
      w[jj] = v[0] * tau[sym_index(0, jj)] + v[1] * tau[sym_index(1, jj)] + v[2] * tau[sym_index(2, jj)];
    // s = g tau + lambda tr(g) I + (mu - c)(g + g^T), g = e_k v^T
    T sm[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) {
        T val = (i == k ? w[jj] + (mu - c) * v[jj] : T(0)) + (jj == k ? (mu - c) * v[i] : T(0));
        if (i == jj) val += lam * v[k];
        sm[i][jj] = val;
      }
    T f[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int d = 0; d < 3; ++d) f[i][d] = W * (sm[i][0] * A[d][0] + sm[i][1] * A[d][1] + sm[i][2] * A[d][2]);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int a1 = a & 1, a2 = (a >> 1) & 1, a3 = a >> 2;
      const T ax = sB[q1 * 2 + a1], ay = sB[q2 * 2 + a2], az = sB[q3 * 2 + a3];
      const T gx = sG[q1 * 2 + a1], gy = sG[q2 * 2 + a2], gz = sG[q3 * 2 + a3];
      const T d0 = gx * ay * az, d1 = ax * gy * az, d2 = ax * ay * gz;
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[a * 3 + i] += d0 * f[i][0] + d1 * f[i][1] + d2 * f[i][2];
    }
  }
  // The matrix is symmetric: store its upper triangle, row-major (entry (r, j), r <= j,
  // at r (47 - r) / 2 + j); column j supplies rows r <= j.
  T *out = K + (int64_t)e * ELMAT_PACKED;
#pragma unroll
  for (int r = 0; r < 24; ++r)
    if (r <= j) out[elmat_index(r, j)] = acc[r];
}

// y_e = K_e x_e for order-1 elements (records for the node-centric assembly).  The
// workgroup's packed matrices (8 x 300 contiguous values) are staged through LDS with
// coalesced loads; thread r then forms row r from the triangle.
template <typename T>
__global__ __launch_bounds__(ELB * 24) void k_elmat_apply(const uint32_t *__restrict__ emap,
                                                          const T *__restrict__ K, const T *__restrict__ x,
                                                          T *__restrict__ ev, int64_t E,
                                                          const double *__restrict__ stop) {
  if (stop && *stop != 0.0) return;  // a stopped PCG (uniform over the grid)
  __shared__ T sx[ELB * 24];
  __shared__ T sK[ELB * ELMAT_PACKED];
  const int t = threadIdx.x, el = t / 24, r = t % 24;
  const int64_t e0 = (int64_t)blockIdx.x * ELB, e = e0 + el;
  const bool live = e < E;
  const int64_t nel = (E - e0) < ELB ? (E - e0) : ELB;
  const T *Kb = K + e0 * ELMAT_PACKED;
  for (int i = t; i < nel * ELMAT_PACKED; i += ELB * 24) sK[i] = Kb[i];
  if (live) {
    const uint32_t w = emap[e * 8 + r / 3];
    const int c = r % 3;
    sx[t] = ((w >> (EMAP_BC_SHIFT + c)) & 1u) ? T(0) : x[(int64_t)(w & EMAP_ID_MASK) * 3 + c];
  }
  __syncthreads();
  if (!live) return;
  const T *Ke = sK + el * ELMAT_PACKED;
  const T *xe = sx + el * 24;
  T acc = 0;
#pragma unroll
  for (int jj = 0; jj < 24; ++jj) acc += Ke[jj < r ? elmat_index(jj, r) : elmat_index(r, jj)] * xe[jj];
  ev[e * 24 + r] = acc;
}

// The order-1 operator assembled into 3 x 3 node blocks, sliced ELL by slot (column
// node cols[j][n], -1 - n past the row's end: a zero block; entry (i, k) at
// vals[j][3 i + k][n] when node_major (each entry of a slot's blocks contiguous over the
// nodes, for a thread per node), else at vals[j][n][3 i + k] (a node's three rows
// contiguous, for a thread per row)).  One
// thread per (slot, row node) sums the block over the elements that hold both nodes,
// in the row node's incidence order (so the result is reproducible), in double, and
// masks it like the matrix-free apply: constrained columns are zero, constrained rows
// identity rows.
template <typename T>
__global__ __launch_bounds__(256) void k_ell_build(bool node_major, int64_t nn, int W, const int32_t *__restrict__ cols,
                                                   const int32_t *__restrict__ off, const int32_t *__restrict__ inc,
                                                   const uint32_t *__restrict__ emap, const T *__restrict__ K,
                                                   T *__restrict__ vals) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)W * nn) return;
  const int j = (int)(t / nn);
  const int64_t n = t - (int64_t)j * nn;
  const int32_t c = cols[t];
  // entry m of this block at blk[m * ms]
  T *blk = node_major ? vals + (int64_t)j * 9 * nn + n : vals + t * 9;
  const int64_t ms = node_major ? nn : 1;
  if (c < 0) {  // padding: a zero block
#pragma unroll
    for (int m = 0; m < 9; ++m) blk[m * ms] = T(0);
    return;
  }
  double a[9];
#pragma unroll
  for (int m = 0; m < 9; ++m) a[m] = 0.0;
  uint32_t rbc = 0, cbc = 0;
  for (int32_t k = off[n]; k < off[n + 1]; ++k) {
    const int32_t rec = inc[k];
    const int64_t e = rec / 8;
    const int la = rec % 8;
    rbc = (emap[rec] >> EMAP_BC_SHIFT) & 7u;
    const T *Ke = K + e * ELMAT_PACKED;
    for (int lb = 0; lb < 8; ++lb) {
      const uint32_t wb = emap[e * 8 + lb];
      if ((int32_t)(wb & EMAP_ID_MASK) != c) continue;
      cbc = (wb >> EMAP_BC_SHIFT) & 7u;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          const int r = la * 3 + i, q = lb * 3 + kk;
          a[i * 3 + kk] += (double)Ke[r <= q ? elmat_index(r, q) : elmat_index(q, r)];
        }
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      double v = ((cbc >> kk) & 1u) ? 0.0 : a[i * 3 + kk];
      if ((rbc >> i) & 1u) v = (c == n && i == kk) ? 1.0 : 0.0;
      blk[(i * 3 + kk) * ms] = (T)v;
    }
}

// ------------------------------------------------------------------------------------
// a11: p-transfer on the same elements (eq. mg_prolong).
// ------------------------------------------------------------------------------------
template <typename T, int PF, int PC>
__global__ __launch_bounds__(QT<PF>::NT) void k_prolong_add(
    const uint32_t *__restrict__ emap_c, const uint32_t *__restrict__ emap_f, const T *__restrict__ xc,
    const T *__restrict__ tab_c, T *__restrict__ yf, int64_t E) {
  constexpr int F3 = PF * PF * PF, C3 = PC * PC * PC, ET = QT<PF>::ET, NQ = ET * F3, NT = QT<PF>::NT;
  constexpr int S = 3 * F3;
  __shared__ T sM[PF * PC];
  __shared__ T lds[2 * ET * S];
  const int tq = threadIdx.x, el = tq / F3, q = tq % F3;
  const int64_t tile = xcd_tile();
  const int64_t e = tile * ET + el;
  const bool live = tq < NQ && e < E;
  load_tables(sM, tab_c, tab_ctof(PF), PF * PC, tq, NT);
  T *a = lds + (live ? el : 0) * S, *b = lds + ET * S + (live ? el : 0) * S;
  uint32_t wf = 0;
  if (live) wf = emap_f[e * F3 + q];
  if (live && q < C3) gather_node(xc, emap_c[e * C3 + q], true, a, q, C3);
  __syncthreads();
  stage<T, PC, PC, PC, 0, PF, false, 3>(a, b, sM, q, live);
  __syncthreads();
  stage<T, PF, PC, PC, 1, PF, false, 3>(b, a, sM, q, live);
  __syncthreads();
  stage<T, PF, PF, PC, 2, PF, false, 3>(a, b, sM, q, live);
  __syncthreads();
  // Every element sharing a fine node interpolates the same value there (the coarse
  // field is continuous); the node's owner element adds it.  No atomics, and the
  // result does not depend on the order in which workgroups run.
  if (live && (wf & EMAP_OWNER)) {
    T *p = yf + (int64_t)(wf & EMAP_ID_MASK) * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (!((wf >> (EMAP_BC_SHIFT + c)) & 1u)) p[c] += b[c * F3 + q];
  }
}

template <typename T, int PF, int PC>
__global__ __launch_bounds__(QT<PF>::NT) void k_restrict(
    const uint32_t *__restrict__ emap_f, const T *__restrict__ rf, const T *__restrict__ tab_c,
    T *__restrict__ ev_c, int64_t E) {
  constexpr int F3 = PF * PF * PF, C3 = PC * PC * PC, ET = QT<PF>::ET, NQ = ET * F3, NT = QT<PF>::NT;
  constexpr int S = 3 * F3;
  __shared__ T sM[PF * PC];
  __shared__ T lds[2 * ET * S];
  const int tq = threadIdx.x, el = tq / F3, q = tq % F3;
  const int64_t tile = xcd_tile();
  const int64_t e = tile * ET + el;
  const bool live = tq < NQ && e < E;
  load_tables(sM, tab_c, tab_ctof(PF), PF * PC, tq, NT);
  T *a = lds + (live ? el : 0) * S, *b = lds + ET * S + (live ? el : 0) * S;
  // Transpose of the owner-written prolongation: each fine node's value enters
  // through its owner element only.
  if (live) {
    const uint32_t w = emap_f[e * F3 + q];
    if (w & EMAP_OWNER) {
      gather_node(rf, w, true, a, q, F3);
    } else {
      a[q] = a[F3 + q] = a[2 * F3 + q] = T(0);
    }
  }
  __syncthreads();
  stage<T, PF, PF, PF, 2, PC, true, 3>(a, b, sM, q, live);
  __syncthreads();
  stage<T, PF, PF, PC, 1, PC, true, 3>(b, a, sM, q, live);
  __syncthreads();
  stage<T, PF, PC, PC, 0, PC, true, 3>(a, b, sM, q, live);
  __syncthreads();
  if (live && q < C3) store_record(ev_c, e, b, q, C3);
}

// ------------------------------------------------------------------------------------
// Strain energy per element (deterministic serial sum over the element's points).
// ------------------------------------------------------------------------------------
template <int P, int Q>
__global__ __launch_bounds__(QT<Q>::NT) void k_energy(const uint32_t *__restrict__ emap,
                                                      const double *__restrict__ u,
                                                      const double *__restrict__ geo,
                                                      const double *__restrict__ tab, double mu0,
                                                      double lam0, const double *__restrict__ mu_e,
                                                      const double *__restrict__ lam_e,
                                                      double *__restrict__ out, int64_t E) {
  using T = double;
  constexpr int Q3 = QT<Q>::Q3, ET = QT<Q>::ET, NQ = QT<Q>::NQ, NT = QT<Q>::NT, P3 = P * P * P;
  constexpr int S0 = 3 * Q3, S1 = 3 * Q3;
  __shared__ T sB[Q * P], sD[Q * Q];
  __shared__ T lds[ET * (S0 + S1)];
  const int tq = threadIdx.x, el = tq / Q3, q = tq % Q3;
  const int64_t tile = xcd_tile();
  const int64_t e = tile * ET + el;
  const bool live = tq < NQ && e < E;
  load_tables(sB, tab, TAB_B, Q * P, tq, NT);
  load_tables(sD, tab, TAB_D, Q * Q, tq, NT);
  T *a = lds + (live ? el : 0) * S0, *b = lds + ET * S0 + (live ? el : 0) * S1;
  if (live && q < P3) {
    const uint32_t node = emap[e * P3 + q] & EMAP_ID_MASK;
#pragma unroll
    for (int c = 0; c < 3; ++c) a[c * P3 + q] = u[(int64_t)node * 3 + c];
  }
  __syncthreads();
  interp<T, P, Q, 3>(a, b, sB, q, live);
  T psi = 0;
  if (live) {
    T G[3][3], D[3][3];
    grad_q<T, Q, 3>(b, sD, q, G);
    const double *g = geo + tile * NGEO * NQ + tq;
    const T W = g[0];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int J = 0; J < 3; ++J) D[k][J] = g[(1 + k * 3 + J) * NQ];
    const T mu = mat_mu(mu0, mu_e, e), lam = mat_mu(lam0, lam_e, e);
    Kin<T> k;
    kinematics(G, D, mu, lam, k);
    T tre = 0;
    for (int i = 0; i < 3; ++i) {
      tre += k.H[i][i];
      for (int j = 0; j < 3; ++j) tre += 0.5 * k.H[i][j] * k.H[i][j];
    }
    psi = W * (0.5 * lam * k.logJ * k.logJ - mu * k.logJ + mu * tre);
  }
  __syncthreads();
  if (live) a[q] = psi;
  __syncthreads();
  if (live && q == 0) {
    T s = 0;
    for (int i = 0; i < Q3; ++i) s += a[i];
    out[e] = s;
  }
}

// ------------------------------------------------------------------------------------
// a16: adjoint (vector-Jacobian product) of the masked residual.
// ------------------------------------------------------------------------------------
template <typename T, int P, int Q, bool STORED>
__global__ __launch_bounds__(QT<Q>::NT) void k_vjp(
    const uint32_t *__restrict__ emap, const double *__restrict__ u, const T *__restrict__ w,
    const double *__restrict__ geo, const T *__restrict__ state, const T *__restrict__ tab,
    double mu0, double lam0, const double *__restrict__ mu_e, const double *__restrict__ lam_e,
    T *__restrict__ ev, double *__restrict__ mub, double *__restrict__ lamb, int64_t E) {
  constexpr int Q3 = QT<Q>::Q3, ET = QT<Q>::ET, NQ = QT<Q>::NQ, NT = QT<Q>::NT, P3 = P * P * P;
  constexpr int NC = STORED ? 3 : 6;
  constexpr int S0 = 9 * Q3, S1 = 6 * Q3;
  __shared__ T sB[Q * P], sD[Q * Q];
  __shared__ T lds[ET * (S0 + S1)];
  const int tq = threadIdx.x, el = tq / Q3, q = tq % Q3;
  const int64_t tile = xcd_tile();
  const int64_t e = tile * ET + el;
  const bool live = tq < NQ && e < E;
  load_tables(sB, tab, TAB_B, Q * P, tq, NT);
  load_tables(sD, tab, TAB_D, Q * Q, tq, NT);
  T *a = lds + (live ? el : 0) * S0, *b = lds + ET * S0 + (live ? el : 0) * S1;
  if (live && q < P3) {
    const uint32_t wd = emap[e * P3 + q];
    const uint32_t node = wd & EMAP_ID_MASK;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a[c * P3 + q] = ((wd >> (EMAP_BC_SHIFT + c)) & 1u) ? T(0) : w[(int64_t)node * 3 + c];
      if (!STORED) a[(3 + c) * P3 + q] = (T)u[(int64_t)node * 3 + c];
    }
  }
  __syncthreads();
  interp<T, P, Q, NC>(a, b, sB, q, live);
  T pm = 0, pl = 0;
  if (live) {
    T G[NC][3], C[3][3], A[3][3], tau[6], c, W;
    grad_q<T, Q, NC>(b, sD, q, G);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) C[i][k] = G[i][k];
    const T mu = (T)mat_mu(mu0, mu_e, e), lam = (T)mat_mu(lam0, lam_e, e);
    T twoe[6];
    double logJ;
    if (STORED) {
      const T *s = state + tile * NSTATE * NQ + tq;
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) A[k][j] = s[(k * 3 + j) * NQ];
#pragma unroll
      for (int m = 0; m < 6; ++m) tau[m] = s[(9 + m) * NQ];
      c = s[15 * NQ];
      // the stored dxi/dx carries sqrt(W): unscale it with the geometry's weight
      W = (T)geo[tile * NGEO * NQ + tq];
      const T rsw = T(1) / (T)sqrt((double)W);
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) A[k][j] *= rsw;
      // tau = 2 mu e + c I and c = lambda log J
#pragma unroll
      for (int m = 0; m < 6; ++m) twoe[m] = (tau[m] - (m < 3 ? c : T(0))) / mu;
      logJ = (double)c / (double)lam;
    } else {
      T Gu[3][3], D[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) Gu[i][k] = G[NC - 3 + i][k];
      const double *g = geo + tile * NGEO * NQ + tq;
      W = (T)g[0];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int J = 0; J < 3; ++J) D[k][J] = (T)g[(1 + k * 3 + J) * NQ];
      Kin<T> k;
      kinematics(Gu, D, mu, lam, k);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) A[i][j] = k.A[i][j];
#pragma unroll
      for (int m = 0; m < 6; ++m) tau[m] = k.tau[m];
      c = k.c;
      logJ = k.logJ;
      for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j)
          twoe[sym_index(i, j)] = k.H[i][j] + k.H[j][i] +
                                  k.H[i][0] * k.H[j][0] + k.H[i][1] * k.H[j][1] + k.H[i][2] * k.H[j][2];
    }
    T f[3][3], M[3][3];
    adjoint_qf(C, A, tau, c, W, mu, lam, f, M);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) a[(i * 3 + k) * Q3 + q] = f[i][k];
    T d = 0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) d += M[i][j] * twoe[sym_index(i, j)];
    pm = W * d;
    pl = W * (T)logJ * (M[0][0] + M[1][1] + M[2][2]);
  }
  __syncthreads();
  // per-element parameter gradients: stage the point values in b, sum serially
  if (live) {
    b[q] = pm;
    b[Q3 + q] = pl;
  }
  grad_t_q<T, Q>(a, sD, q, b + 2 * Q3, live);
  __syncthreads();
  if (live && q == 0) {
    T sm = 0, sl = 0;
    for (int i = 0; i < Q3; ++i) {
      sm += b[i];
      sl += b[Q3 + i];
    }
    if (mub) mub[e] = (double)sm;
    if (lamb) lamb[e] = (double)sl;
  }
  // move the transposed-gradient result to the front of b for interp_t
  T tmp[3];
  if (live) {
#pragma unroll
    for (int c2 = 0; c2 < 3; ++c2) tmp[c2] = b[2 * Q3 + c2 * Q3 + q];
  }
  __syncthreads();
  if (live) {
#pragma unroll
    for (int c2 = 0; c2 < 3; ++c2) b[c2 * Q3 + q] = tmp[c2];
  }
  __syncthreads();
  interp_t<T, P, Q, 3>(b, a, sB, q, live);
  if (live && q < P3) store_record(ev, e, a, q, P3);
}

// Geometric factors out of the tiled layout into [E][10][Q^3].
template <int Q>
__global__ void k_export_geo(const double *__restrict__ geo, double *__restrict__ out, int64_t E) {
  constexpr int Q3 = QT<Q>::Q3, ET = QT<Q>::ET, NQ = QT<Q>::NQ;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = E * NGEO * Q3;
  if (i >= total) return;
  const int64_t e = i / (NGEO * Q3);
  const int f = (int)((i / Q3) % NGEO), q = (int)(i % Q3);
  const int64_t tile = e / ET;
  const int el = (int)(e % ET);
  out[i] = geo[(tile * NGEO + f) * NQ + el * Q3 + q];
}

// Internal element map with Dirichlet bits.
__global__ void k_build_emap(const int32_t *__restrict__ en, const uint8_t *__restrict__ mask,
                             uint32_t *__restrict__ emap, int64_t n, int64_t N,
                             unsigned *__restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t node = en[i];
  if (node < 0 || node >= N) {
    atomicOr(flags, 4u);
    emap[i] = 0;
    return;
  }
  uint32_t w = (uint32_t)node;
  if (mask) {
    for (int c = 0; c < 3; ++c)
      if (mask[(int64_t)node * 3 + c]) w |= 1u << (EMAP_BC_SHIFT + c);
  }
  emap[i] = w;
}

// Node-centric assembly: y[n] = sum of the node's element records, in the fixed order
// of its incidence list; constrained components take `src` (or zero).
template <typename T>
__global__ __launch_bounds__(256) void k_assemble(int64_t N, const int32_t *__restrict__ off,
                                                  const int32_t *__restrict__ inc, const T *__restrict__ ev,
                                                  const uint8_t *__restrict__ mask, const T *__restrict__ src,
                                                  T fill, T *__restrict__ y) {
  // One node per thread; consecutive node ranges stay on one XCD (see xcd_tile), so
  // the records of neighbouring nodes, which share elements, meet in the same L2.
  const int64_t n = xcd_tile() * blockDim.x + threadIdx.x;
  if (n < N) {
    const int32_t k0 = off[n], k1 = off[n + 1];
    T a0 = 0, a1 = 0, a2 = 0;
    for (int32_t k = k0; k < k1; ++k) {
      const T *p = ev + (int64_t)inc[k] * 3;
      a0 += p[0];
      a1 += p[1];
      a2 += p[2];
    }
    if (mask) {
      const uint8_t *m = mask + n * 3;
      if (m[0]) a0 = src ? src[n * 3] : fill;
      if (m[1]) a1 = src ? src[n * 3 + 1] : fill;
      if (m[2]) a2 = src ? src[n * 3 + 2] : fill;
    }
    T *o = y + n * 3;
    o[0] = a0;
    o[1] = a1;
    o[2] = a2;
  }
}

// The same node sums with the output staged in LDS and written by the workgroup in
// contiguous nontemporal sweeps (256 consecutive nodes = 768 consecutive values), so
// every store instruction covers whole cache lines.
template <typename T>
__global__ __launch_bounds__(256) void k_assemble_staged(int64_t N, const int32_t *__restrict__ off,
                                                         const int32_t *__restrict__ inc, const T *__restrict__ ev,
                                                         const uint8_t *__restrict__ mask, const T *__restrict__ src,
                                                         T fill, T *__restrict__ y) {
  __shared__ T buf[3 * 256];
  // consecutive node ranges stay on one XCD (see xcd_tile): neighbouring nodes share
  // elements, so their records meet in the same L2
  const int64_t n0 = xcd_tile() * 256, n = n0 + threadIdx.x;
  if (n < N) {
    const int32_t k0 = off[n], k1 = off[n + 1];
    T a0 = 0, a1 = 0, a2 = 0;
    for (int32_t k = k0; k < k1; ++k) {
      const T *p = ev + (int64_t)inc[k] * 3;
      a0 += p[0];
      a1 += p[1];
      a2 += p[2];
    }
    if (mask) {
      const uint8_t *m = mask + n * 3;
      if (m[0]) a0 = src ? src[n * 3] : fill;
      if (m[1]) a1 = src ? src[n * 3 + 1] : fill;
      if (m[2]) a2 = src ? src[n * 3 + 2] : fill;
    }
    buf[3 * threadIdx.x] = a0;
    buf[3 * threadIdx.x + 1] = a1;
    buf[3 * threadIdx.x + 2] = a2;
  }
  __syncthreads();
  const int nv = 3 * (int)((N - n0) < 256 ? (N - n0) : 256);
  T *o = y + n0 * 3;
  for (int d = threadIdx.x; d < nv; d += 256) __builtin_nontemporal_store(buf[d], o + d);
}

// The same assembly fused with the partial dot product p . y of the assembled result
// and the direction p (= src), one partial per workgroup (fixed tree): the Jacobi-PCG
// step needs p^T A p right after A p.
template <typename T>
__global__ __launch_bounds__(256) void k_assemble_dot(int64_t N, const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ inc, const T *__restrict__ ev,
                                                      const uint8_t *__restrict__ mask, const T *__restrict__ src,
                                                      T *__restrict__ y, double *__restrict__ partial,
                                                      const double *__restrict__ stop) {
  if (stop && *stop != 0.0) return;  // a stopped PCG (uniform over the grid)
  __shared__ double red[256];
  const int64_t tile = xcd_tile();
  const int64_t n = tile * blockDim.x + threadIdx.x;
  double pq = 0.0;
  if (n < N) {
    const int32_t k0 = off[n], k1 = off[n + 1];
    T a[3] = {0, 0, 0};
    for (int32_t k = k0; k < k1; ++k) {
      const T *p = ev + (int64_t)inc[k] * 3;
      a[0] += p[0];
      a[1] += p[1];
      a[2] += p[2];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (mask && mask[n * 3 + c]) a[c] = src[n * 3 + c];
      y[n * 3 + c] = a[c];
      pq += (double)src[n * 3 + c] * (double)a[c];
    }
  }
  red[threadIdx.x] = pq;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < (unsigned)w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[tile] = red[0];
}

inline unsigned grid1d(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// y = assembled element records of `op`; constrained components take src (or `fill`).
template <typename T>
hipError_t assemble(const hpmg_op_s &op, const T *src, T *y, hipStream_t s, T fill = T(0)) {
  int64_t g = (op.N + 255) / 256;
  if (g < 1) g = 1;
  if (sweep_records<T>(op.P))
    k_assemble_staged<T><<<(unsigned)g, 256, 0, s>>>(op.N, op.csr_off, op.csr_inc, (const T *)op.evec, op.mask, src,
                                                      fill, y);
  else
    k_assemble<T><<<(unsigned)g, 256, 0, s>>>(op.N, op.csr_off, op.csr_inc, (const T *)op.evec, op.mask, src, fill,
                                               y);
  return hipGetLastError();
}

// The first record of every node (incidence lists are in record order) owns it.
__global__ void k_mark_owners(int64_t N, const int32_t *__restrict__ off, const int32_t *__restrict__ inc,
                              uint32_t *__restrict__ emap) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N && off[n] < off[n + 1]) emap[inc[off[n]]] |= EMAP_OWNER;
}

// ------------------------------------------------------------------------------------
// (P, Q) dispatch.
// ------------------------------------------------------------------------------------
#define HPMG_PQ_LIST(X) \
  X(2, 2) X(2, 3) X(2, 4) X(2, 5) X(3, 3) X(3, 4) X(3, 5) X(4, 4) X(4, 5) X(5, 5) X(5, 6)

#define HPMG_PP_LIST(X) X(3, 2) X(4, 2) X(5, 2) X(4, 3) X(5, 3) X(5, 4)

}  // namespace

bool supported_pq(int P, int Q) {
#define X(p, q) if (P == p && Q == q) return true;
  HPMG_PQ_LIST(X)
#undef X
  return false;
}

static bool supported_pp(int Pf, int Pc) {
#define X(f, c) if (Pf == f && Pc == c) return true;
  HPMG_PP_LIST(X)
#undef X
  return false;
}

hipError_t launch_build_emap(const hpmg_op_s &op, hipStream_t s) {
  const int64_t n = op.E * op.P * op.P * op.P;
  k_build_emap<<<grid1d(n, 256), 256, 0, s>>>(op.elem_nodes, op.mask, op.emap, n, op.N, op.flags);
  return hipGetLastError();
}

hipError_t launch_mark_owners(const hpmg_op_s &op, hipStream_t s) {
  k_mark_owners<<<grid1d(op.N, 256), 256, 0, s>>>(op.N, op.csr_off, op.csr_inc, op.emap);
  return hipGetLastError();
}

hipError_t launch_qdata(const hpmg_op_s &op, const double *X, hipStream_t s) {
#define X(p, q)                                                                              \
  if (op.P == p && op.Q == q) {                                                              \
    k_qdata<p, q><<<(unsigned)op.tiles, QT<q>::NT, 0, s>>>(op.emap, X, op.tab64, op.geo, op.flags, op.E); \
    return hipGetLastError();                                                                \
  }
  HPMG_PQ_LIST(X)
#undef X
  return hipErrorInvalidValue;
}

// Residual: the element kernel writes element records, the node-centric assembly pass
// sums them (deterministic).
hipError_t launch_residual(const hpmg_op_s &op, const double *u, double *r, bool store, hipStream_t s) {
#define X(p, q)                                                                                  \
  if (op.P == p && op.Q == q) {                                                                  \
    lines_launch<double, p, q, 4>((unsigned)op.tiles, s, keep_records<double>(op.E, p), op.emap, u,            \
                                  (const double *)nullptr, op.geo, (const double *)nullptr, op.tab64, op.mu,      \
                                  op.lam, op.mu_e, op.lam_e, (double *)op.evec, op.E, (const double *)nullptr,    \
                                  store ? op.state64 : nullptr, op.flags, (const double *)nullptr);               \
    hipError_t e = hipGetLastError();                                                            \
    if (e != hipSuccess) return e;                                                               \
    return assemble<double>(op, nullptr, r, s);                                                  \
  }
  HPMG_PQ_LIST(X)
#undef X
  return hipErrorInvalidValue;
}

template <typename T, int P, int Q>
static hipError_t jacobian_pq(const hpmg_op_s &op, const hpmg_op_s &f, int mode, const double *u, const T *du,
                              T *ev, const double *stop, hipStream_t s) {
  const T *state = std::is_same<T, double>::value ? (const T *)f.state64 : (const T *)f.state32;
  const T *tab = std::is_same<T, double>::value ? (const T *)op.tab64 : (const T *)op.tab32;
  const bool keep = keep_records<T>(op.E, P);
  const unsigned g = (unsigned)op.tiles;
  if constexpr (std::is_same<T, double>::value) {
    if (mode == HPMG_INITIAL_NATIVE || mode == HPMG_INITIAL_TUNED || mode == HPMG_CURRENT_20) {
      if (mode == HPMG_INITIAL_NATIVE)
        lines_launch<T, P, Q, 1>(g, s, keep, op.emap, du, nullptr, op.geo, op.sinit, tab, op.mu, op.lam, op.mu_e,
                                 op.lam_e, ev, op.E, nullptr, nullptr, nullptr, nullptr);
      else if (mode == HPMG_INITIAL_TUNED)
        lines_launch<T, P, Q, 2>(g, s, keep, op.emap, du, nullptr, op.geo, op.sinit, tab, op.mu, op.lam, op.mu_e,
                                 op.lam_e, ev, op.E, nullptr, nullptr, nullptr, nullptr);
      else
        lines_launch<T, P, Q, 3>(g, s, keep, op.emap, du, nullptr, op.geo, op.sinit, tab, op.mu, op.lam, op.mu_e,
                                 op.lam_e, ev, op.E, nullptr, nullptr, nullptr, nullptr);
      return hipGetLastError();
    }
  }
  if (mode == HPMG_STORED) {
    lines_launch<T, P, Q, 0>(g, s, keep, op.emap, du, state, nullptr, nullptr, tab, f.mu, f.lam, f.mu_e, f.lam_e,
                             ev, op.E, stop, nullptr, nullptr, nullptr);
  } else {
    lines_launch<T, P, Q, 5>(g, s, keep, op.emap, du, (const T *)nullptr, op.geo, (const double *)nullptr, tab,
                             op.mu, op.lam, op.mu_e, op.lam_e, ev, op.E, (const double *)nullptr,
                             (double *)nullptr, (unsigned *)nullptr, u);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t assemble_or_dot(const hpmg_op_s &op, const T *du, T *y, double *pq, const double *stop,
                                  hipStream_t s) {
  if (!pq) return assemble<T>(op, du, y, s);
  k_assemble_dot<T><<<grid1d(op.N, 256), 256, 0, s>>>(op.N, op.csr_off, op.csr_inc, (const T *)op.evec, op.mask,
                                                      du, y, pq, stop);
  return hipGetLastError();
}

// pq != NULL: the assembly also writes per-workgroup partials of du . y (ceil(N / 256)).
// stop != NULL: the stored-mode kernels return at once while *stop != 0.
template <typename T>
static hipError_t jacobian_t(const hpmg_op_s &op, int mode, const double *u, const T *du, T *y, hipStream_t s,
                             double *pq = nullptr, const double *stop = nullptr) {
  const hpmg_op_s &f = op.fine ? *op.fine : op;
  T *ev = (T *)op.evec;
  const int tprec = std::is_same<T, double>::value ? HPMG_F64 : HPMG_F32;
  if (mode == HPMG_STORED && op.P == 2 && op.elmat && op.elmat_prec == tprec &&
      op.elmat_version == f.state_version) {
    k_elmat_apply<T><<<grid1d(op.E, ELB), ELB * 24, 0, s>>>(op.emap, (const T *)op.elmat, du, ev, op.E, stop);
    hipError_t e2 = hipGetLastError();
    if (e2 != hipSuccess) return e2;
    return assemble_or_dot<T>(op, du, y, pq, stop, s);
  }
  hipError_t e = hipErrorInvalidValue;
#define X(p, q) \
  if (op.P == p && op.Q == q) e = jacobian_pq<T, p, q>(op, f, mode, u, du, ev, stop, s);
  HPMG_PQ_LIST(X)
#undef X
  if (e != hipSuccess) return e;
  return assemble_or_dot<T>(op, du, y, pq, stop, s);
}

hipError_t launch_jacobian_dot(const hpmg_op_s &op, int prec, const void *du, void *y, double *pq,
                               const double *stop, hipStream_t s) {
  if (prec == HPMG_F64)
    return jacobian_t<double>(op, HPMG_STORED, nullptr, (const double *)du, (double *)y, s, pq, stop);
  return jacobian_t<float>(op, HPMG_STORED, nullptr, (const float *)du, (float *)y, s, pq, stop);
}

hipError_t launch_jacobian(const hpmg_op_s &op, int prec, int mode, const double *u, const void *du,
                           void *y, hipStream_t s) {
  if (prec == HPMG_F64) return jacobian_t<double>(op, mode, u, (const double *)du, (double *)y, s);
  return jacobian_t<float>(op, mode, u, (const float *)du, (float *)y, s);
}

hipError_t launch_diagonal(const hpmg_op_s &op, int prec, void *diag, hipStream_t s) {
  const hpmg_op_s &f = op.fine ? *op.fine : op;
  if (prec == HPMG_F64) {
#define X(p, q)                                                                                    \
  if (op.P == p && op.Q == q) {                                                                    \
    k_diagonal<double, p, q><<<(unsigned)op.tiles, QT<q>::NT, 0, s>>>(                              \
        op.emap, f.state64, op.tab64, f.mu, f.lam, f.mu_e, f.lam_e, (double *)op.evec, op.E);    \
    hipError_t e = hipGetLastError();                                                              \
    return e != hipSuccess ? e : assemble<double>(op, nullptr, (double *)diag, s, 1.0);            \
  }
    HPMG_PQ_LIST(X)
#undef X
  } else {
#define X(p, q)                                                                                   \
  if (op.P == p && op.Q == q) {                                                                   \
    k_diagonal<float, p, q><<<(unsigned)op.tiles, QT<q>::NT, 0, s>>>(                              \
        op.emap, f.state32, op.tab32, f.mu, f.lam, f.mu_e, f.lam_e, (float *)op.evec, op.E);     \
    hipError_t e = hipGetLastError();                                                             \
    return e != hipSuccess ? e : assemble<float>(op, nullptr, (float *)diag, s, 1.0f);            \
  }
    HPMG_PQ_LIST(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t launch_prolong_add(const hpmg_op_s &c, const hpmg_op_s &f, int prec, const void *xc, void *yf,
                              hipStream_t s) {
  const unsigned grid = grid1d(f.E, elems_per_tile(f.P));
#define X(pf, pc)                                                                                     \
  if (f.P == pf && c.P == pc) {                                                                       \
    if (prec == HPMG_F64)                                                                             \
      k_prolong_add<double, pf, pc><<<grid, QT<pf>::NT, 0, s>>>(c.emap, f.emap, (const double *)xc,    \
                                                                c.tab64, (double *)yf, f.E);          \
    else                                                                                              \
      k_prolong_add<float, pf, pc><<<grid, QT<pf>::NT, 0, s>>>(c.emap, f.emap, (const float *)xc,      \
                                                               c.tab32, (float *)yf, f.E);            \
    return hipGetLastError();                                                                         \
  }
  HPMG_PP_LIST(X)
#undef X
  (void)supported_pp;
  return hipErrorInvalidValue;
}

hipError_t launch_restrict(const hpmg_op_s &f, const hpmg_op_s &c, int prec, const void *rf, void *rc,
                           hipStream_t s) {
  const unsigned grid = grid1d(f.E, elems_per_tile(f.P));
#define X(pf, pc)                                                                                    \
  if (f.P == pf && c.P == pc) {                                                                      \
    if (prec == HPMG_F64) {                                                                          \
      k_restrict<double, pf, pc><<<grid, QT<pf>::NT, 0, s>>>(f.emap, (const double *)rf, c.tab64,     \
                                                             (double *)c.evec, f.E);                 \
      hipError_t e = hipGetLastError();                                                              \
      return e != hipSuccess ? e : assemble<double>(c, nullptr, (double *)rc, s);                    \
    }                                                                                                \
    k_restrict<float, pf, pc><<<grid, QT<pf>::NT, 0, s>>>(f.emap, (const float *)rf, c.tab32,         \
                                                          (float *)c.evec, f.E);                      \
    hipError_t e = hipGetLastError();                                                                \
    return e != hipSuccess ? e : assemble<float>(c, nullptr, (float *)rc, s);                        \
  }
  HPMG_PP_LIST(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_energy(const hpmg_op_s &op, const double *u, double *psi, hipStream_t s) {
#define X(p, q)                                                                                  \
  if (op.P == p && op.Q == q) {                                                                  \
    k_energy<p, q><<<(unsigned)op.tiles, QT<q>::NT, 0, s>>>(op.emap, u, op.geo, op.tab64, op.mu, op.lam, \
                                                            op.mu_e, op.lam_e, op.scratch, op.E); \
    hipError_t e = hipGetLastError();                                                            \
    if (e != hipSuccess) return e;                                                               \
    return launch_sum(op.E, op.scratch, op.scratch + op.E, psi, s);                              \
  }
  HPMG_PQ_LIST(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_body_load(const hpmg_op_s &op, const double *g, double *f_ext, hipStream_t s) {
#define X(p, q)                                                                                      \
  if (op.P == p && op.Q == q) {                                                                      \
    k_body_load<p, q><<<(unsigned)op.tiles, QT<q>::NT, 0, s>>>(op.geo, op.tab64, g[0], g[1], g[2], op.evec, \
                                                               op.E);                                \
    hipError_t e = hipGetLastError();                                                                \
    return e != hipSuccess ? e : assemble<double>(op, nullptr, f_ext, s);                            \
  }
  HPMG_PQ_LIST(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_traction_load(const hpmg_op_s &op, const double *coords, int64_t nf, const int32_t *face_elem,
                                const int32_t *face_id, const double *t, double *rec, int32_t *rec_node,
                                hipStream_t s) {
#define X(p, q)                                                                                      \
  if (op.P == p && op.Q == q) {                                                                      \
    k_traction_load<p, q><<<grid1d(nf, 64), 64, 0, s>>>(coords, op.elem_nodes, face_elem, face_id,        \
                                                         op.tab64,                                    \
                                                         t[0], t[1], t[2], nf, op.E, rec, rec_node,   \
                                                         op.flags);                                  \
    return hipGetLastError();                                                                        \
  }
  HPMG_PQ_LIST(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_assemble_csr(int64_t N, const int32_t *off, const int32_t *inc, const double *rec,
                               const uint8_t *mask, double *y, hipStream_t s) {
  k_assemble<double><<<grid1d(N, 256), 256, 0, s>>>(N, off, inc, rec, mask, nullptr, 0.0, y);
  return hipGetLastError();
}

hipError_t launch_state_initial(const hpmg_op_s &op, const double *u, hipStream_t s) {
#define X(p, q)                                                                                      \
  if (op.P == p && op.Q == q) {                                                                      \
    k_state_initial<p, q><<<(unsigned)op.tiles, QT<q>::NT, 0, s>>>(op.emap, u, op.geo, op.tab64, op.mu, \
                                                                   op.lam, op.mu_e, op.lam_e, op.sinit, \
                                                                   op.flags, op.E);                  \
    return hipGetLastError();                                                                        \
  }
  HPMG_PQ_LIST(X)
#undef X
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t vjp_t(const hpmg_op_s &op, int mode, const double *u, const T *w, T *ub, double *mub,
                        double *lamb, hipStream_t s) {
  T *ev = (T *)op.evec;
  const T *state = std::is_same<T, double>::value ? (const T *)op.state64 : (const T *)op.state32;
  const T *tab = std::is_same<T, double>::value ? (const T *)op.tab64 : (const T *)op.tab32;
#define X(p, q)                                                                                      \
  if (op.P == p && op.Q == q) {                                                                      \
    if (mode == HPMG_STORED)                                                                         \
      k_vjp<T, p, q, true><<<(unsigned)op.tiles, QT<q>::NT, 0, s>>>(op.emap, u, w, op.geo, state, tab,  \
                                                                    op.mu, op.lam, op.mu_e, op.lam_e, \
                                                                    ev, mub, lamb, op.E);            \
    else                                                                                             \
      k_vjp<T, p, q, false><<<(unsigned)op.tiles, QT<q>::NT, 0, s>>>(op.emap, u, w, op.geo, state, tab, \
                                                                     op.mu, op.lam, op.mu_e, op.lam_e, \
                                                                     ev, mub, lamb, op.E);           \
    hipError_t e = hipGetLastError();                                                                \
    if (e != hipSuccess) return e;                                                                   \
    /* unmasked assembly: constrained columns of u_bar are kept */                                   \
    k_assemble<T><<<grid1d(op.N, 256), 256, 0, s>>>(op.N, op.csr_off, op.csr_inc, ev, nullptr, nullptr, \
                                                    T(0), ub);                                       \
    return hipGetLastError();                                                                        \
  }
  HPMG_PQ_LIST(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_vjp(const hpmg_op_s &op, int prec, int mode, const double *u, const void *w, void *ub,
                      double *mub, double *lamb, hipStream_t s) {
  if (prec == HPMG_F64) return vjp_t<double>(op, mode, u, (const double *)w, (double *)ub, mub, lamb, s);
  return vjp_t<float>(op, mode, u, (const float *)w, (float *)ub, mub, lamb, s);
}

hipError_t launch_elmat_build(const hpmg_op_s &op, int prec, hipStream_t s) {
  const hpmg_op_s &f = op.fine ? *op.fine : op;  // the operator holding the linearisation
  const unsigned g = grid1d(op.E, ELB);
#define X(q)                                                                                          \
  if (op.Q == q) {                                                                                    \
    if (prec == HPMG_F64)                                                                             \
      k_elmat_build<double, q><<<g, ELB * 24, 0, s>>>(f.state64, op.tab64, f.mu, f.lam, f.mu_e, f.lam_e, \
                                                      op.elmat, op.E);                               \
    else                                                                                              \
      k_elmat_build<float, q><<<g, ELB * 24, 0, s>>>(f.state32, op.tab32, f.mu, f.lam, f.mu_e, f.lam_e,  \
                                                     (float *)op.elmat, op.E);                        \
    return hipGetLastError();                                                                         \
  }
  X(2) X(3) X(4) X(5)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_ell_build(const hpmg_op_s &op, int prec, bool node_major, int64_t W, const int32_t *cols,
                            void *vals,
                            hipStream_t s) {
  if (op.P != 2 || !op.elmat || op.elmat_prec != prec) return hipErrorInvalidValue;
  const unsigned g = grid1d(W * op.N, 256);
  if (prec == HPMG_F64)
    k_ell_build<double><<<g, 256, 0, s>>>(node_major, op.N, (int)W, cols, op.csr_off, op.csr_inc, op.emap,
                                          (const double *)op.elmat, (double *)vals);
  else
    k_ell_build<float><<<g, 256, 0, s>>>(node_major, op.N, (int)W, cols, op.csr_off, op.csr_inc, op.emap,
                                         (const float *)op.elmat, (float *)vals);
  return hipGetLastError();
}

hipError_t launch_export_qdata(const hpmg_op_s &op, double *out, hipStream_t s) {
  const int64_t total = op.E * NGEO * op.Q * op.Q * op.Q;
  switch (op.Q) {
    case 2: k_export_geo<2><<<grid1d(total, 256), 256, 0, s>>>(op.geo, out, op.E); break;
    case 3: k_export_geo<3><<<grid1d(total, 256), 256, 0, s>>>(op.geo, out, op.E); break;
    case 4: k_export_geo<4><<<grid1d(total, 256), 256, 0, s>>>(op.geo, out, op.E); break;
    case 5: k_export_geo<5><<<grid1d(total, 256), 256, 0, s>>>(op.geo, out, op.E); break;
    case 6: k_export_geo<6><<<grid1d(total, 256), 256, 0, s>>>(op.geo, out, op.E); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace hpmg
