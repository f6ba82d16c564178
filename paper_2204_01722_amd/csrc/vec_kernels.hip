// Vector kernels for the Krylov and multigrid drivers: boundary-condition fills,
// precision casts, fused axpy-type updates, and deterministic FP64 reductions.
//
// Reductions run on a fixed grid (RED_BLOCKS workgroups of 256 threads): each thread
// accumulates a grid-strided slice in double, a 64-lane wavefront reduces with
// cross-lane shuffles, the four wavefronts of a workgroup combine through LDS, and a
// single workgroup sums the RED_BLOCKS partials in a fixed tree.  The result does not
// depend on timing, so repeated runs are bitwise identical.
#include "common.h"

namespace hpmg {
namespace {

constexpr int BS = 256;

inline unsigned grid_for(int64_t n) {
  int64_t g = (n + BS - 1) / BS;
  if (g < 1) g = 1;
  if (g > 65535 * 16) g = 65535 * 16;
  return (unsigned)g;
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

template <typename T>
__global__ void k_init_bc(int64_t nn, const uint8_t *__restrict__ mask, const T *__restrict__ x,
                          T *__restrict__ y) {
  GRID_STRIDE(i, 3 * nn) { y[i] = (mask && x && mask[i]) ? x[i] : T(0); }
}

__global__ void k_cast_d2f(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
  GRID_STRIDE(i, n) { b[i] = (float)a[i]; }
}

__global__ void k_cast_f2d(int64_t n, const float *__restrict__ a, double *__restrict__ b) {
  GRID_STRIDE(i, n) { b[i] = (double)a[i]; }
}

template <typename T>
__global__ void k_axpby(int64_t n, T a, const T *__restrict__ x, T b, T *__restrict__ y) {
  GRID_STRIDE(i, n) { y[i] = a * x[i] + b * y[i]; }
}

template <typename T>
__global__ void k_waxpby(int64_t n, T a, const T *__restrict__ x, T b, const T *__restrict__ y,
                         T *__restrict__ w) {
  GRID_STRIDE(i, n) { w[i] = a * x[i] + b * y[i]; }
}

template <typename T>
__global__ void k_cg_update(int64_t n, T alpha, const T *__restrict__ p, const T *__restrict__ q,
                            T *__restrict__ x, const T *__restrict__ rin, T *__restrict__ rout) {
  GRID_STRIDE(i, n) {
    x[i] += alpha * p[i];
    rout[i] = rin[i] - alpha * q[i];
  }
}

template <typename T>
__global__ void k_recip(int64_t n, T *__restrict__ x) {
  GRID_STRIDE(i, n) { x[i] = T(1) / x[i]; }
}

// r = Dinv (b - Ax); d = r / theta; x = d (Ax == null: zero initial guess) or x += d.
template <typename T>
__global__ void k_cheb_first(int64_t n, const T *__restrict__ dinv, const T *__restrict__ b,
                             const T *__restrict__ Ax, T *__restrict__ r, T *__restrict__ d,
                             T *__restrict__ x, T inv_theta) {
  GRID_STRIDE(i, n) {
    const T ri = dinv[i] * (Ax ? b[i] - Ax[i] : b[i]);
    const T di = ri * inv_theta;
    r[i] = ri;
    d[i] = di;
    x[i] = Ax ? x[i] + di : di;
  }
}

// r -= Dinv A d; d = c1 d + c2 r; x += d.
template <typename T>
__global__ void k_cheb_step(int64_t n, const T *__restrict__ dinv, T *__restrict__ r,
                            const T *__restrict__ Ad, T *__restrict__ d, T *__restrict__ x, T c1, T c2) {
  GRID_STRIDE(i, n) {
    const T ri = r[i] - dinv[i] * Ad[i];
    const T di = c1 * d[i] + c2 * ri;
    r[i] = ri;
    d[i] = di;
    x[i] += di;
  }
}

// ---- reductions -------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block sum of NV values per thread into out[v * gridDim.x + blockIdx.x].
template <int NV>
__device__ __forceinline__ void block_store(double (&v)[NV], double *__restrict__ partial) {
  __shared__ double s[NV][BS / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double w = wave_sum(v[k]);
    if (lane == 0) s[k][wid] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double t = 0.0;
      for (int j = 0; j < BS / 64; ++j) t += s[k][j];
      partial[k * gridDim.x + blockIdx.x] = t;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_dot_partial(int64_t n, const T *__restrict__ x,
                                                    const T *__restrict__ y, double *__restrict__ partial) {
  double v[1] = {0.0};
  GRID_STRIDE(i, n) { v[0] += (double)x[i] * (double)y[i]; }
  block_store<1>(v, partial);
}

template <typename T>
__global__ __launch_bounds__(BS) void k_dot2_partial(int64_t n, const T *__restrict__ x,
                                                     const T *__restrict__ y, const T *__restrict__ z,
                                                     double *__restrict__ partial) {
  double v[2] = {0.0, 0.0};
  GRID_STRIDE(i, n) {
    v[0] += (double)x[i] * (double)y[i];
    v[1] += (double)z[i] * (double)z[i];
  }
  block_store<2>(v, partial);
}

template <typename T>
__global__ __launch_bounds__(BS) void k_jacobi_dot_partial(int64_t n, const T *__restrict__ dinv,
                                                           const T *__restrict__ r, T *__restrict__ z,
                                                           double *__restrict__ partial) {
  double v[2] = {0.0, 0.0};
  GRID_STRIDE(i, n) {
    const T ri = r[i];
    const T zi = dinv[i] * ri;
    z[i] = zi;
    v[0] += (double)ri * (double)zi;
    v[1] += (double)ri * (double)ri;
  }
  block_store<2>(v, partial);
}

template <typename T>
__global__ __launch_bounds__(BS) void k_dot_pair_partial(int64_t n, const T *__restrict__ z,
                                                         const T *__restrict__ a, const T *__restrict__ b,
                                                         double *__restrict__ partial) {
  double v[2] = {0.0, 0.0};
  GRID_STRIDE(i, n) {
    const double zi = (double)z[i];
    v[0] += zi * (double)a[i];
    v[1] += zi * (double)b[i];
  }
  block_store<2>(v, partial);
}

__global__ __launch_bounds__(BS) void k_sum_partial(int64_t n, const double *__restrict__ x,
                                                    double *__restrict__ partial) {
  double v[1] = {0.0};
  GRID_STRIDE(i, n) { v[0] += x[i]; }
  block_store<1>(v, partial);
}

// One workgroup: out[k] = sum of partial[k * nb .. k * nb + nb) in a fixed tree.
__global__ __launch_bounds__(RED_BLOCKS) void k_final(const double *__restrict__ partial, int nb, int nv,
                                                      double *__restrict__ out) {
  __shared__ double s[RED_BLOCKS];
  for (int k = 0; k < nv; ++k) {
    s[threadIdx.x] = threadIdx.x < (unsigned)nb ? partial[k * nb + threadIdx.x] : 0.0;
    __syncthreads();
    for (int w = RED_BLOCKS / 2; w > 0; w >>= 1) {
      if (threadIdx.x < (unsigned)w) s[threadIdx.x] += s[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = s[0];
    __syncthreads();
  }
}

// NV sums of partial[v * stride + 0 .. nb) by the whole workgroup in a fixed order
// (strided per-thread sums, a wave butterfly, the waves in order); every thread gets
// the results.
template <int NV>
__device__ __forceinline__ void block_reduce_fixed_n(const double *__restrict__ partial, int nb, int stride,
                                                     double (&out)[NV]) {
  __shared__ double s[NV][BS / 64];
  double t[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) t[v] = 0.0;
  for (int i = threadIdx.x; i < nb; i += BS)
#pragma unroll
    for (int v = 0; v < NV; ++v) t[v] += partial[v * stride + i];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    t[v] = wave_sum(t[v]);
    if (lane == 0) s[v][wid] = t[v];
  }
  __syncthreads();
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < BS / 64; ++w) r += s[v][w];
    out[v] = r;
  }
  __syncthreads();
}

__device__ __forceinline__ double block_reduce_fixed(const double *__restrict__ partial, int nb) {
  double o[1];
  block_reduce_fixed_n<1>(partial, nb, 0, o);
  return o[0];
}

// Fused Jacobi-PCG iteration (four launches: the operator's element kernel, its
// assembly fused with the partials of p.q, update2 and dir2).  The curvature p.q arrives
// as workgroup partials of the fused assembly; rz alternates between scalar slots 8 and
// 9 so that no workgroup overwrites a value another one still reads.  The convergence
// test runs on the device: dir2 raises sc[SC_STOP], after which every kernel of later
// iterations returns at once, so the host can queue many iterations and read the
// scalars rarely.
__global__ void k_pcg_begin(double *__restrict__ sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc[8] = sc[2];
    sc[SC_RR0] = sc[3];
    sc[5] = 0.0;
    sc[SC_STOP] = 0.0;
    sc[SC_COUNT] = 0.0;
  }
}

// update2: alpha = rz / pq, x += alpha p (skipped when x is null: the eigenvalue estimate
// needs only the coefficients), r -= alpha q, z = D^-1 r, partials of r.z, r.r.
template <typename T>
__global__ __launch_bounds__(BS) void k_pcg_update2(int64_t n, double *__restrict__ sc, int parity, int nb_pq,
                                                    const double *__restrict__ pq_partial,
                                                    const T *__restrict__ p, const T *__restrict__ q,
                                                    T *__restrict__ x, T *__restrict__ r,
                                                    const T *__restrict__ dinv, T *__restrict__ z,
                                                    double *__restrict__ partial, double *__restrict__ alpha_rec) {
  if (sc[SC_STOP] != 0.0) return;
  const double pq = block_reduce_fixed(pq_partial, nb_pq);
  const double alpha = pq > 0.0 ? sc[8 + parity] / pq : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[1] = pq;
    if (!(pq > 0.0)) sc[5] = 1.0;
    if (alpha_rec) *alpha_rec = alpha;
  }
  const T a = (T)alpha;
  double v[2] = {0.0, 0.0};
  GRID_STRIDE(i, n) {
    if (x) x[i] += a * p[i];
    const T ri = r[i] - a * q[i];
    r[i] = ri;
    const T zi = dinv[i] * ri;
    z[i] = zi;
    v[0] += (double)ri * (double)zi;
    v[1] += (double)ri * (double)ri;
  }
  block_store<2>(v, partial);
}

// dir2: rz_new and r.r from the partials, beta = rz_new / rz, p = z + beta p; counts the
// iteration and decides whether to stop.
template <typename T>
__global__ __launch_bounds__(BS) void k_pcg_dir2(int64_t n, double *__restrict__ sc, int parity,
                                                 const double *__restrict__ partial, const T *__restrict__ z,
                                                 T *__restrict__ p, double rtol2, double *__restrict__ beta_rec) {
  if (sc[SC_STOP] != 0.0) return;
  double red2[2];
  block_reduce_fixed_n<2>(partial, RED_BLOCKS, RED_BLOCKS, red2);
  const double rz_new = red2[0], rr = red2[1];
  const double rz = sc[8 + parity];
  const bool broke = sc[5] != 0.0;
  const double beta = rz != 0.0 ? rz_new / rz : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (broke) {
      sc[SC_STOP] = 1.0;
    } else {
      sc[8 + (parity ^ 1)] = rz_new;
      sc[2] = rz_new;
      sc[3] = rr;
      sc[SC_COUNT] += 1.0;
      if (beta_rec) *beta_rec = beta;
      if (rtol2 >= 0.0 && rr <= rtol2 * sc[SC_RR0]) sc[SC_STOP] = 1.0;
    }
  }
  if (broke) return;
  const T b = (T)beta;
  GRID_STRIDE(i, n) { p[i] = z[i] + b * p[i]; }
}

__global__ __launch_bounds__(BS) void k_fcg_update(int64_t n, double *__restrict__ sc, int it,
                                                   const double *__restrict__ p, const double *__restrict__ q,
                                                   double *__restrict__ x, const double *__restrict__ r,
                                                   double *__restrict__ rn, double *__restrict__ partial) {
  const double pq = sc[FCG_PQ], rz = sc[FCG_RZ + (it & 1)];
  const bool brk = !(pq > 0.0) || !isfinite(rz);
  const double a = brk ? 0.0 : rz / pq;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[FCG_BRK] = brk ? 1.0 : 0.0;
    sc[FCG_ALPHA] = a;
  }
  double v[1] = {0.0};
  GRID_STRIDE(i, n) {
    x[i] += a * p[i];
    const double ri = r[i] - a * q[i];
    rn[i] = ri;
    v[0] += ri * ri;
  }
  block_store<1>(v, partial);
}

__global__ __launch_bounds__(BS) void k_fcg_dir(int64_t n, double *__restrict__ sc, int it,
                                                const double *__restrict__ z, double *__restrict__ p) {
  const double zrn = sc[FCG_ZRN], rz = sc[FCG_RZ + (it & 1)];
  const double beta = (zrn - sc[FCG_ZR]) / rz;
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[FCG_RZ + ((it + 1) & 1)] = zrn;
  GRID_STRIDE(i, n) { p[i] = z[i] + beta * p[i]; }
}

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Jacobi-PCG iteration `it` on an assembled operator held as 3 x 3 blocks in sliced ELL
// (slot j of node n: column node cols[j][n], or -1 - n for padding past the row's end,
// whose block is zero), replacing the element kernel, the fused assembly and dir2 of the
// four-launch iteration.  Prologue (it > 0, every workgroup alike): r.z and r.r of
// iteration it - 1 from the update's partials, beta, the stopping test (as in dir2; the
// count is set, not incremented, so a repeated prologue changes nothing).  The body
// forms the new direction p = z + beta p_old on the fly for every column node read,
// with one fused multiply-add, so all threads that need a node's p agree bit for bit;
// the row's own value goes to p_new (p_old and p_new alternate between two buffers),
// q = A p to y, and the partial of p.q to pq_part[workgroup].  WC > 0 fixes the width
// at compile time, so the loads of several slots can be issued together.  nn = 0 runs
// the prologue alone.  Two bodies and block layouts (node_major; by default by size):
//  * rows: a thread per scalar row, the three rows of a node on neighbouring lanes (they
//    read the same column nodes); block entry (i, k) at vals[j][n][3 i + k].  Three
//    times the threads of the other form: the faster one while the coarse level is small
//    (per iteration at 21^3 nodes 23.4 against 34.5 us in FP64).
//  * nodes: a thread per node and its three rows; entry (i, k) at vals[j][3 i + k][n],
//    so each of a block's nine loads is one contiguous run over the workgroup's nodes.
//    The faster one once the block matrix streams from HBM (per iteration at 61^3 nodes
//    154.9 against 202.6 us in FP64, 68.5 against 105.6 us in FP32); equal at 41^3.

// The prologue; false: the iteration stops (every thread of the grid agrees).
__device__ __forceinline__ bool ell_prologue(double *__restrict__ sc, const double *__restrict__ partial, int it,
                                             double rtol2, double &beta) {
  beta = 0.0;
  if (it == 0) return true;
  double red2[2];
  block_reduce_fixed_n<2>(partial, RED_BLOCKS, RED_BLOCKS, red2);
  const double rz_new = red2[0], rr = red2[1];
  const double rz = sc[8 + ((it - 1) & 1)];
  const bool broke = sc[5] != 0.0;
  const bool conv = !broke && rtol2 >= 0.0 && rr <= rtol2 * sc[SC_RR0];
  beta = rz != 0.0 ? rz_new / rz : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (!broke) {
      sc[8 + (it & 1)] = rz_new;
      sc[2] = rz_new;
      sc[3] = rr;
      sc[SC_COUNT] = (double)it;
    }
    if (broke || conv) sc[SC_STOP] = 1.0;
  }
  return !(broke || conv);
}

template <typename T, int WC>
__global__ __launch_bounds__(BS) void k_ell_pcg_rows(int64_t nn, int W, const int32_t *__restrict__ cols,
                                                     const T *__restrict__ vals, const T *__restrict__ z,
                                                     const T *__restrict__ p_old, T *__restrict__ p_new,
                                                     T *__restrict__ y, double *__restrict__ sc,
                                                     const double *__restrict__ partial, int it, double rtol2,
                                                     double *__restrict__ pq_part) {
  if (sc[SC_STOP] != 0.0) return;
  double beta;
  if (!ell_prologue(sc, partial, it, rtol2, beta) || nn == 0) return;
  const bool first = it == 0;
  const T b = (T)beta;
  double v[1] = {0.0};
  const int64_t t = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (t < 3 * nn) {
    const int64_t n = t / 3;
    const int i = (int)(t - 3 * n);
    // direction value of node c, component k (the same expression wherever it is formed)
    auto pdir = [&](int64_t c, int k) { return first ? z[c * 3 + k] : fma_t(b, p_old[c * 3 + k], z[c * 3 + k]); };
    auto slot = [&](int j, int32_t c0) {
      const int64_t c = c0 < 0 ? -1 - (int64_t)c0 : (int64_t)c0;
      const T *A = vals + ((int64_t)j * nn + n) * 9 + 3 * i;
      return A[0] * pdir(c, 0) + A[1] * pdir(c, 1) + A[2] * pdir(c, 2);
    };
    T acc = 0;
    if constexpr (WC > 0) {
      // all column ids first (one wait), then the blocks in groups whose loads are
      // issued together (9 in FP32, 3 in FP64, as the registers allow)
      constexpr int UR = sizeof(T) == 4 ? 9 : 3;
      static_assert(WC % UR == 0, "width must be a multiple of the unroll");
      int32_t cj[WC];
#pragma unroll
      for (int j = 0; j < WC; ++j) cj[j] = cols[(int64_t)j * nn + n];
      for (int j0 = 0; j0 < WC; j0 += UR) {
        T part[UR];
#pragma unroll
        for (int u = 0; u < UR; ++u) part[u] = slot(j0 + u, cj[j0 + u]);
#pragma unroll
        for (int u = 0; u < UR; ++u) acc += part[u];
      }
    } else {
      for (int j = 0; j < W; ++j) acc += slot(j, cols[(int64_t)j * nn + n]);
    }
    const T pn = pdir(n, i);
    p_new[t] = pn;
    y[t] = acc;
    v[0] = (double)pn * (double)acc;
  }
  block_store<1>(v, pq_part);
}

template <typename T, int WC>
__global__ __launch_bounds__(BS) void k_ell_pcg_nodes(int64_t nn, int W, const int32_t *__restrict__ cols,
                                                      const T *__restrict__ vals, const T *__restrict__ z,
                                                      const T *__restrict__ p_old, T *__restrict__ p_new,
                                                      T *__restrict__ y, double *__restrict__ sc,
                                                      const double *__restrict__ partial, int it, double rtol2,
                                                      double *__restrict__ pq_part) {
  if (sc[SC_STOP] != 0.0) return;
  double beta;
  if (!ell_prologue(sc, partial, it, rtol2, beta) || nn == 0) return;
  const bool first = it == 0;
  const T b = (T)beta;
  double v[1] = {0.0};
  const int64_t n = (int64_t)blockIdx.x * BS + threadIdx.x;
  if (n < nn) {
    auto pdir = [&](int64_t c, int k) { return first ? z[c * 3 + k] : fma_t(b, p_old[c * 3 + k], z[c * 3 + k]); };
    // the block of slot j (column node c0) times the direction at that node
    auto slot = [&](int j, int32_t c0, T (&part)[3]) {
      const int64_t c = c0 < 0 ? -1 - (int64_t)c0 : (int64_t)c0;
      T pd[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) pd[k] = pdir(c, k);
      const T *A = vals + (int64_t)j * 9 * nn + n;
#pragma unroll
      for (int i = 0; i < 3; ++i)
        part[i] = A[(3 * i) * nn] * pd[0] + A[(3 * i + 1) * nn] * pd[1] + A[(3 * i + 2) * nn] * pd[2];
    };
    T acc[3] = {0, 0, 0};
    if constexpr (WC > 0) {
      constexpr int UR = sizeof(T) == 4 ? 3 : 1;
      static_assert(WC % UR == 0, "width must be a multiple of the unroll");
      int32_t cj[WC];
#pragma unroll
      for (int j = 0; j < WC; ++j) cj[j] = cols[(int64_t)j * nn + n];
      for (int j0 = 0; j0 < WC; j0 += UR) {
        T part[UR][3];
#pragma unroll
        for (int u = 0; u < UR; ++u) slot(j0 + u, cj[j0 + u], part[u]);
#pragma unroll
        for (int u = 0; u < UR; ++u)
#pragma unroll
          for (int i = 0; i < 3; ++i) acc[i] += part[u][i];
      }
    } else {
      for (int j = 0; j < W; ++j) {
        T part[3];
        slot(j, cols[(int64_t)j * nn + n], part);
#pragma unroll
        for (int i = 0; i < 3; ++i) acc[i] += part[i];
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T pn = pdir(n, i);
      p_new[n * 3 + i] = pn;
      y[n * 3 + i] = acc[i];
      v[0] += (double)pn * (double)acc[i];
    }
  }
  block_store<1>(v, pq_part);
}

}  // namespace

hipError_t launch_fcg_update(int64_t n, double *sc, int it, const double *p, const double *q, double *x,
                             const double *r, double *rn, double *partial, hipStream_t s) {
  k_fcg_update<<<RED_BLOCKS, BS, 0, s>>>(n, sc, it, p, q, x, r, rn, partial);
  k_final<<<1, RED_BLOCKS, 0, s>>>(partial, RED_BLOCKS, 1, sc + FCG_RR);
  return hipGetLastError();
}

hipError_t launch_fcg_dir(int64_t n, double *sc, int it, const double *z, double *p, hipStream_t s) {
  k_fcg_dir<<<grid_for(n), BS, 0, s>>>(n, sc, it, z, p);
  return hipGetLastError();
}

hipError_t launch_pcg_begin(double *sc, hipStream_t s) {
  k_pcg_begin<<<1, 64, 0, s>>>(sc);
  return hipGetLastError();
}

int ell_pcg_blocks(int64_t nn, bool node_major) {
  return node_major ? (int)((nn + BS - 1) / BS) : (int)((3 * nn + BS - 1) / BS);
}

hipError_t launch_ell_pcg_apply(int prec, bool nodes, int64_t nn, int W, const int32_t *cols, const void *vals,
                                const void *z,
                                const void *p_old, void *p_new, void *y, double *sc, const double *partial, int it,
                                double rtol2, double *pq_part, hipStream_t s) {
  const unsigned g = nn > 0 ? (unsigned)ell_pcg_blocks(nn, nodes) : 1u;
#define ELL_LAUNCH(TT, WC)                                                                                    \
  do {                                                                                                        \
    if (nodes)                                                                                                \
      k_ell_pcg_nodes<TT, WC><<<g, BS, 0, s>>>(nn, W, cols, (const TT *)vals, (const TT *)z, (const TT *)p_old, \
                                               (TT *)p_new, (TT *)y, sc, partial, it, rtol2, pq_part);          \
    else                                                                                                      \
      k_ell_pcg_rows<TT, WC><<<g, BS, 0, s>>>(nn, W, cols, (const TT *)vals, (const TT *)z, (const TT *)p_old,  \
                                              (TT *)p_new, (TT *)y, sc, partial, it, rtol2, pq_part);           \
  } while (0)
  // 27: every node of a hexahedral mesh interior
  if (prec == HPMG_F64) {
    if (W == 27)
      ELL_LAUNCH(double, 27);
    else
      ELL_LAUNCH(double, 0);
  } else {
    if (W == 27)
      ELL_LAUNCH(float, 27);
    else
      ELL_LAUNCH(float, 0);
  }
#undef ELL_LAUNCH
  return hipGetLastError();
}

hipError_t launch_pcg_update2(int prec, int64_t n, double *sc, int parity, int nb_pq, const double *pq_partial,
                              const void *p, const void *q, void *x, void *r, const void *dinv, void *z,
                              double *partial, double *alpha_rec, hipStream_t s) {
  if (prec == HPMG_F64)
    k_pcg_update2<double><<<RED_BLOCKS, BS, 0, s>>>(n, sc, parity, nb_pq, pq_partial, (const double *)p,
                                                    (const double *)q, (double *)x, (double *)r,
                                                    (const double *)dinv, (double *)z, partial, alpha_rec);
  else
    k_pcg_update2<float><<<RED_BLOCKS, BS, 0, s>>>(n, sc, parity, nb_pq, pq_partial, (const float *)p,
                                                   (const float *)q, (float *)x, (float *)r, (const float *)dinv,
                                                   (float *)z, partial, alpha_rec);
  return hipGetLastError();
}

hipError_t launch_pcg_dir2(int prec, int64_t n, double *sc, int parity, const double *partial, const void *z,
                           void *p, double rtol2, double *beta_rec, hipStream_t s) {
  if (prec == HPMG_F64)
    k_pcg_dir2<double><<<RED_BLOCKS, BS, 0, s>>>(n, sc, parity, partial, (const double *)z, (double *)p, rtol2,
                                                 beta_rec);
  else
    k_pcg_dir2<float><<<RED_BLOCKS, BS, 0, s>>>(n, sc, parity, partial, (const float *)z, (float *)p, rtol2,
                                                beta_rec);
  return hipGetLastError();
}


size_t prec_size(int prec) { return prec == HPMG_F64 ? sizeof(double) : sizeof(float); }

#define DISPATCH(prec, CALL_D, CALL_F) \
  do {                                 \
    if ((prec) == HPMG_F64) {          \
      CALL_D;                          \
    } else {                           \
      CALL_F;                          \
    }                                  \
    return hipGetLastError();          \
  } while (0)

hipError_t launch_init_bc(int prec, int64_t nn, const uint8_t *mask, const void *x, void *y, hipStream_t s) {
  DISPATCH(prec, (k_init_bc<double><<<grid_for(3 * nn), BS, 0, s>>>(nn, mask, (const double *)x, (double *)y)),
           (k_init_bc<float><<<grid_for(3 * nn), BS, 0, s>>>(nn, mask, (const float *)x, (float *)y)));
}

__global__ void k_inject(int64_t nc, const int32_t *__restrict__ map, const double *__restrict__ uf,
                         double *__restrict__ uc) {
  GRID_STRIDE(i, 3 * nc) { uc[i] = uf[(int64_t)map[i / 3] * 3 + i % 3]; }
}

hipError_t launch_inject(int64_t nc, const int32_t *map, const double *uf, double *uc, hipStream_t s) {
  k_inject<<<grid_for(3 * nc), BS, 0, s>>>(nc, map, uf, uc);
  return hipGetLastError();
}

hipError_t launch_cast_state(int64_t n, const double *a, float *b, hipStream_t s) {
  k_cast_d2f<<<grid_for(n), BS, 0, s>>>(n, a, b);
  return hipGetLastError();
}

hipError_t launch_cast(int64_t n, int to_prec, const void *x, void *y, hipStream_t s) {
  if (to_prec == HPMG_F32)
    k_cast_d2f<<<grid_for(n), BS, 0, s>>>(n, (const double *)x, (float *)y);
  else
    k_cast_f2d<<<grid_for(n), BS, 0, s>>>(n, (const float *)x, (double *)y);
  return hipGetLastError();
}

hipError_t launch_axpby(int prec, int64_t n, double a, const void *x, double b, void *y, hipStream_t s) {
  DISPATCH(prec, (k_axpby<double><<<grid_for(n), BS, 0, s>>>(n, a, (const double *)x, b, (double *)y)),
           (k_axpby<float><<<grid_for(n), BS, 0, s>>>(n, (float)a, (const float *)x, (float)b, (float *)y)));
}

hipError_t launch_waxpby(int prec, int64_t n, double a, const void *x, double b, const void *y, void *w,
                         hipStream_t s) {
  DISPATCH(prec,
           (k_waxpby<double><<<grid_for(n), BS, 0, s>>>(n, a, (const double *)x, b, (const double *)y, (double *)w)),
           (k_waxpby<float><<<grid_for(n), BS, 0, s>>>(n, (float)a, (const float *)x, (float)b, (const float *)y,
                                                       (float *)w)));
}

hipError_t launch_cg_update(int prec, int64_t n, double alpha, const void *p, const void *q, void *x,
                            const void *rin, void *rout, hipStream_t s) {
  DISPATCH(prec,
           (k_cg_update<double><<<grid_for(n), BS, 0, s>>>(n, alpha, (const double *)p, (const double *)q,
                                                           (double *)x, (const double *)rin, (double *)rout)),
           (k_cg_update<float><<<grid_for(n), BS, 0, s>>>(n, (float)alpha, (const float *)p, (const float *)q,
                                                          (float *)x, (const float *)rin, (float *)rout)));
}

hipError_t launch_recip(int prec, int64_t n, void *x, hipStream_t s) {
  DISPATCH(prec, (k_recip<double><<<grid_for(n), BS, 0, s>>>(n, (double *)x)),
           (k_recip<float><<<grid_for(n), BS, 0, s>>>(n, (float *)x)));
}

hipError_t launch_cheb_first(int prec, int64_t n, const void *dinv, const void *b, const void *Ax, void *r,
                             void *d, void *x, double inv_theta, hipStream_t s) {
  DISPATCH(prec,
           (k_cheb_first<double><<<grid_for(n), BS, 0, s>>>(n, (const double *)dinv, (const double *)b,
                                                            (const double *)Ax, (double *)r, (double *)d,
                                                            (double *)x, inv_theta)),
           (k_cheb_first<float><<<grid_for(n), BS, 0, s>>>(n, (const float *)dinv, (const float *)b,
                                                           (const float *)Ax, (float *)r, (float *)d,
                                                           (float *)x, (float)inv_theta)));
}

hipError_t launch_cheb_step(int prec, int64_t n, const void *dinv, void *r, const void *Ad, void *d, void *x,
                            double c1, double c2, hipStream_t s) {
  DISPATCH(prec,
           (k_cheb_step<double><<<grid_for(n), BS, 0, s>>>(n, (const double *)dinv, (double *)r,
                                                           (const double *)Ad, (double *)d, (double *)x, c1, c2)),
           (k_cheb_step<float><<<grid_for(n), BS, 0, s>>>(n, (const float *)dinv, (float *)r, (const float *)Ad,
                                                          (float *)d, (float *)x, (float)c1, (float)c2)));
}

hipError_t launch_dot(int prec, int64_t n, const void *x, const void *y, double *partial, double *out,
                      hipStream_t s) {
  if (prec == HPMG_F64)
    k_dot_partial<double><<<RED_BLOCKS, BS, 0, s>>>(n, (const double *)x, (const double *)y, partial);
  else
    k_dot_partial<float><<<RED_BLOCKS, BS, 0, s>>>(n, (const float *)x, (const float *)y, partial);
  k_final<<<1, RED_BLOCKS, 0, s>>>(partial, RED_BLOCKS, 1, out);
  return hipGetLastError();
}

hipError_t launch_dot2(int prec, int64_t n, const void *x, const void *y, const void *z, double *partial,
                       double *out, hipStream_t s) {
  if (prec == HPMG_F64)
    k_dot2_partial<double><<<RED_BLOCKS, BS, 0, s>>>(n, (const double *)x, (const double *)y, (const double *)z,
                                                     partial);
  else
    k_dot2_partial<float><<<RED_BLOCKS, BS, 0, s>>>(n, (const float *)x, (const float *)y, (const float *)z,
                                                    partial);
  k_final<<<1, RED_BLOCKS, 0, s>>>(partial, RED_BLOCKS, 2, out);
  return hipGetLastError();
}

hipError_t launch_jacobi_dot(int prec, int64_t n, const void *dinv, const void *r, void *z, double *partial,
                             double *out, hipStream_t s) {
  if (prec == HPMG_F64)
    k_jacobi_dot_partial<double><<<RED_BLOCKS, BS, 0, s>>>(n, (const double *)dinv, (const double *)r,
                                                           (double *)z, partial);
  else
    k_jacobi_dot_partial<float><<<RED_BLOCKS, BS, 0, s>>>(n, (const float *)dinv, (const float *)r, (float *)z,
                                                          partial);
  k_final<<<1, RED_BLOCKS, 0, s>>>(partial, RED_BLOCKS, 2, out);
  return hipGetLastError();
}

hipError_t launch_dot_pair(int prec, int64_t n, const void *z, const void *a, const void *b, double *partial,
                           double *out, hipStream_t s) {
  if (prec == HPMG_F64)
    k_dot_pair_partial<double><<<RED_BLOCKS, BS, 0, s>>>(n, (const double *)z, (const double *)a,
                                                         (const double *)b, partial);
  else
    k_dot_pair_partial<float><<<RED_BLOCKS, BS, 0, s>>>(n, (const float *)z, (const float *)a, (const float *)b,
                                                        partial);
  k_final<<<1, RED_BLOCKS, 0, s>>>(partial, RED_BLOCKS, 2, out);
  return hipGetLastError();
}

hipError_t launch_sum(int64_t n, const double *x, double *partial, double *out, hipStream_t s) {
  k_sum_partial<<<RED_BLOCKS, BS, 0, s>>>(n, x, partial);
  k_final<<<1, RED_BLOCKS, 0, s>>>(partial, RED_BLOCKS, 1, out);
  return hipGetLastError();
}

}  // namespace hpmg
