// Sum-factorised FP64 kernels: the same volume, surface and trace
// contractions as the dense operators, evaluated through the collapsed
// tensor structure of the semi-nodal basis
//   phi_ijk(a, b, c) = l^k_i(a) l^k_j(b) g_k(c),  g_k = h^k P^{(2k+3,0)}_{N-k}(c),
// on the tensor cubature (a_p, b_m, c_r) (the lower-cost evaluation of volume
// integrals that Section 4.4 proposes).  Derivatives in (r, s, t):
//   d/dr phi = l'(a) l(b) h^(k-1) P,  d/ds phi = l(a) l'(b) h^(k-1) P,
//   d/dt phi = l l g_k' + (1+a)/2 d/dr phi + (1+b)/2 d/ds phi.
// Results equal the dense contractions up to rounding order.
#include <hip/hip_runtime.h>

#include "context.hpp"
#include "flux.hpp"
#include "geom.hpp"

namespace dgpyr {
namespace {

constexpr int kThreads = 256;

template <int N>
struct SfDim {
  static constexpr int n1 = N + 1;
  static constexpr int Np = (N + 1) * (N + 2) * (2 * N + 3) / 6;
  static constexpr int Nfq = n1 * n1;
  static constexpr int Nfc = 5 * Nfq;
  static constexpr int E = N <= 2 ? 16 : N <= 4 ? 8 : N <= 6 ? 4 : 2;  // elements per block
};

__device__ __forceinline__ int kofs(int k) { return k * (k + 1) * (2 * k + 1) / 6; }

// Traces at every face point of every element into T[K][Nfc][4].  One work
// item per (element, face, p) evaluates the (N+1) points of column p.
template <int N>
__global__ __launch_bounds__(kThreads) void k_trace_sf(const double* __restrict__ U,
                                                       double* __restrict__ T, SfOps sf,
                                                       int64_t K) {
  using D = SfDim<N>;
  constexpr int n1 = D::n1;
  __shared__ double sU[D::E * 4 * D::Np];
  const int64_t e0 = (int64_t)blockIdx.x * D::E;
  const int ne = (int)((K - e0) < D::E ? (K - e0) : D::E);
  for (int x = threadIdx.x; x < ne * 4 * D::Np; x += kThreads) sU[x] = U[e0 * 4 * D::Np + x];
  __syncthreads();
  for (int x = threadIdx.x; x < ne * 5 * n1; x += kThreads) {
    const int le = x / (5 * n1), rem = x - le * 5 * n1;
    const int f = rem / n1, p = rem - f * n1;
    const double* su = sU + le * 4 * D::Np;
    double out[n1][4];
#pragma unroll
    for (int m = 0; m < n1; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) out[m][v] = 0.0;
#pragma unroll
    for (int k = 0; k <= N; ++k) {
      const double* La_p = sf.La + (k * n1 + p) * n1;  // l^k_i(x_p)
      const double* Le_s = sf.Le + (k * 2 + ((f == 2 || f == 4) ? 1 : 0)) * n1;
      const int ob = kofs(k);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double* u = su + v * D::Np + ob;
        if (f == 0) {
          // base: sum_j l_j(b_m) sum_i l_i(a_p) u_ijk, then g_k(-1)
          double X[n1];
#pragma unroll
          for (int j = 0; j <= k; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i <= k; ++i) acc += La_p[i] * u[j * (k + 1) + i];
            X[j] = acc;
          }
          const double gb = sf.Gb[k];
#pragma unroll
          for (int m = 0; m < n1; ++m) {
            const double* La_m = sf.La + (k * n1 + m) * n1;
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j <= k; ++j) acc += La_m[j] * X[j];
            out[m][v] += gb * acc;
          }
        } else {
          // a = -1/+1 (f = 1/2): sum_j l_j(b_p) sum_i l_i(+-1) u_ijk
          // b = -1/+1 (f = 3/4): sum_j l_j(+-1) sum_i l_i(a_p) u_ijk
          double Y = 0.0;
#pragma unroll
          for (int j = 0; j <= k; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i <= k; ++i)
              acc += (f <= 2 ? Le_s[i] : La_p[i]) * u[j * (k + 1) + i];
            Y += (f <= 2 ? La_p[j] : Le_s[j]) * acc;
          }
#pragma unroll
          for (int m = 0; m < n1; ++m) out[m][v] += sf.Gf[m * n1 + k] * Y;
        }
      }
    }
    double* o = T + ((e0 + le) * D::Nfc + f * D::Nfq + p) * 4;
#pragma unroll
    for (int m = 0; m < n1; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) o[m * n1 * 4 + v] = out[m][v];
  }
}

// Per (p, m) column: a0_k = sum_j l_j(b_m) sum_i l_i(a_p) u_ijk,
// aa_k (with l'(a_p)), ab_k (with l'(b_m)).
template <int N>
__device__ __forceinline__ void column_factors(const double* __restrict__ u, const SfOps& sf, int p,
                                               int m, double* a0, double* aa, double* ab) {
  constexpr int n1 = N + 1;
#pragma unroll
  for (int k = 0; k <= N; ++k) {
    const double* La_p = sf.La + (k * n1 + p) * n1;
    const double* Da_p = sf.Da + (k * n1 + p) * n1;
    const double* La_m = sf.La + (k * n1 + m) * n1;
    const double* Da_m = sf.Da + (k * n1 + m) * n1;
    const double* uk = u + kofs(k);
    double s0 = 0.0, sa = 0.0, sb = 0.0;
#pragma unroll
    for (int j = 0; j <= k; ++j) {
      double x = 0.0, xd = 0.0;
#pragma unroll
      for (int i = 0; i <= k; ++i) {
        const double uv = uk[j * (k + 1) + i];
        x += La_p[i] * uv;
        xd += Da_p[i] * uv;
      }
      s0 += La_m[j] * x;
      sb += Da_m[j] * x;
      sa += La_m[j] * xd;
    }
    a0[k] = s0;
    aa[k] = sa;
    ab[k] = sb;
  }
}

// Fused stage: volume term, surface term, inverse mass and (MODE 1) the RK
// stage, sum-factorised.  Phase A: one work item per (element, p, m) column
// evaluates the derivatives along c, applies the FP64 metric (constant along
// the column), and folds the projection's c-sum and the base-face lift into
// B_f[k][m][p] = sum_r g_k(c_r) Q_f(p, m, r) + g_k(-1) F_f(p, m).  Phase A':
// one work item per (element, triangle, p) folds the triangle fluxes along c:
// C_f[k][p] = sum_m g_k(c_m) F_f(p, m).  Phase C: one work item per basis
// function finishes the a and b sums and applies M^-1 and the RK update.
template <int N, int MODE>
__global__ __launch_bounds__(kThreads) void k_stage_sf(const double* U,
                                                       const double* __restrict__ T, SfOps sf,
                                                       DevOps ops, DevMesh mesh, double* out,
                                                       double* R, double ra, double rb, double dt) {
  using D = SfDim<N>;
  constexpr int n1 = D::n1, Np = D::Np;
  __shared__ double sU[D::E * 4 * Np];
  __shared__ double sB[D::E * 4 * n1 * n1 * n1];  // [e][f][k][m][p]
  __shared__ double sC[D::E * 4 * 4 * n1 * n1];   // [e][face-1][f][k][p]
  __shared__ double sX[D::E * 16];
  const int64_t e0 = (int64_t)blockIdx.x * D::E;
  const int ne = (int)((mesh.K - e0) < D::E ? (mesh.K - e0) : D::E);
  for (int x = threadIdx.x; x < ne * 4 * Np; x += kThreads) sU[x] = U[e0 * 4 * Np + x];
  for (int x = threadIdx.x; x < ne * 16; x += kThreads) sX[x] = mesh.verts[e0 * 16 + x];
  __syncthreads();

  // Phase A: volume + base face, per (element, p, m)
  for (int x = threadIdx.x; x < ne * n1 * n1; x += kThreads) {
    const int le = x / (n1 * n1), pm = x - le * n1 * n1;
    const int p = pm % n1, m = pm / n1;
    const int64_t e = e0 + le;
    const double* su = sU + le * 4 * Np;
    const double* xv = sX + le * 16;
    const double ap = ops.xg[p], bm = ops.xg[m];
    double adj[9], J;
    pyr_metric(xv, ap, bm, adj, &J);
    const double wab = 0.25 * ops.wf[pm];  // wg[p] wg[m] / 4 (base-face weights)
    const double ha = 0.5 * (1.0 + ap), hb = 0.5 * (1.0 + bm);
    double Bf[4][n1];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int k = 0; k < n1; ++k) Bf[v][k] = 0.0;
    double a0[n1], aa[n1], ab[n1];
    // pressure: Q_u_k = w sum_rho adj[rho][k] d_rho p
    column_factors<N>(su, sf, p, m, a0, aa, ab);
#pragma unroll
    for (int r = 0; r < n1; ++r) {
      double dr = 0.0, ds = 0.0, dtp = 0.0;
#pragma unroll
      for (int k = 0; k <= N; ++k) {
        dr += sf.Gt[r * n1 + k] * aa[k];
        ds += sf.Gt[r * n1 + k] * ab[k];
        dtp += sf.Gp[r * n1 + k] * a0[k];
      }
      const double dtt = dtp + ha * dr + hb * ds;
      const double w = wab * sf.wc[r];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        const double q = w * (adj[kk] * dr + adj[3 + kk] * ds + adj[6 + kk] * dtt);
#pragma unroll
        for (int k = 0; k <= N; ++k) Bf[1 + kk][k] += sf.G[r * n1 + k] * q;
      }
    }
    // velocity components: Q_p = w sum_k sum_rho adj[rho][k] d_rho u_k
    double Qp[n1];
#pragma unroll
    for (int r = 0; r < n1; ++r) Qp[r] = 0.0;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      column_factors<N>(su + (1 + kk) * Np, sf, p, m, a0, aa, ab);
#pragma unroll
      for (int r = 0; r < n1; ++r) {
        double dr = 0.0, ds = 0.0, dtp = 0.0;
#pragma unroll
        for (int k = 0; k <= N; ++k) {
          dr += sf.Gt[r * n1 + k] * aa[k];
          ds += sf.Gt[r * n1 + k] * ab[k];
          dtp += sf.Gp[r * n1 + k] * a0[k];
        }
        const double dtt = dtp + ha * dr + hb * ds;
        Qp[r] += adj[kk] * dr + adj[3 + kk] * ds + adj[6 + kk] * dtt;
      }
    }
#pragma unroll
    for (int r = 0; r < n1; ++r) {
      const double w = wab * sf.wc[r];
#pragma unroll
      for (int k = 0; k <= N; ++k) Bf[0][k] += sf.G[r * n1 + k] * (w * Qp[r]);
    }
    // base face (c = -1) point (p, m): lift weight g_k(-1)
    if (e < mesh.K) {
      double F[4];
      face_flux<D::Nfq>(T, ops, mesh, xv, e, pm, F);
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int k = 0; k <= N; ++k) Bf[v][k] += sf.Gb[k] * F[v];
    }
    double* sb = sB + le * 4 * n1 * n1 * n1;
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int k = 0; k <= N; ++k) sb[((v * n1 + k) * n1 + m) * n1 + p] = Bf[v][k];
  }

  // Phase A': triangle faces, per (element, face, p)
  for (int x = threadIdx.x; x < ne * 4 * n1; x += kThreads) {
    const int le = x / (4 * n1), rem = x - le * 4 * n1;
    const int ft = rem / n1, p = rem - ft * n1;  // ft = face - 1
    const int64_t e = e0 + le;
    const double* xv = sX + le * 16;
    double Cf[4][n1];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int k = 0; k < n1; ++k) Cf[v][k] = 0.0;
#pragma unroll
    for (int m = 0; m < n1; ++m) {
      double F[4];
      face_flux<D::Nfq>(T, ops, mesh, xv, e, (ft + 1) * D::Nfq + p + n1 * m, F);
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int k = 0; k <= N; ++k) Cf[v][k] += sf.Gf[m * n1 + k] * F[v];
    }
    double* sc = sC + (le * 4 + ft) * 4 * n1 * n1;
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int k = 0; k <= N; ++k) sc[(v * n1 + k) * n1 + p] = Cf[v][k];
  }
  __syncthreads();

  // Phase C: per (element, basis function)
  for (int x = threadIdx.x; x < ne * Np; x += kThreads) {
    const int le = x / Np, n = x - le * Np;
    const int64_t e = e0 + le;
    // (i, j, k) of n in the canonical order
    int k = 0;
    while (kofs(k + 1) <= n) ++k;
    const int rem = n - kofs(k), j = rem / (k + 1), i = rem - j * (k + 1);
    const double* sb = sB + le * 4 * n1 * n1 * n1;
    const double* sc = sC + le * 4 * 4 * n1 * n1;
    const double* La_k = sf.La + k * n1 * n1;  // [p][i]
    const double lm1_i = sf.Le[(k * 2 + 0) * n1 + i], lp1_i = sf.Le[(k * 2 + 1) * n1 + i];
    const double lm1_j = sf.Le[(k * 2 + 0) * n1 + j], lp1_j = sf.Le[(k * 2 + 1) * n1 + j];
    double acc[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double* b = sb + (v * n1 + k) * n1 * n1;
      double z = 0.0;
#pragma unroll
      for (int m = 0; m < n1; ++m) {
        double y = 0.0;
#pragma unroll
        for (int p = 0; p < n1; ++p) y += La_k[p * n1 + i] * b[m * n1 + p];
        z += La_k[m * n1 + j] * y;
      }
      // triangles a = -1, a = +1 (sum over the b-like edge coordinate p)
      const double* c1 = sc + ((0 * 4 + v) * n1 + k) * n1;
      const double* c2 = sc + ((1 * 4 + v) * n1 + k) * n1;
      const double* c3 = sc + ((2 * 4 + v) * n1 + k) * n1;
      const double* c4 = sc + ((3 * 4 + v) * n1 + k) * n1;
      double t1 = 0.0, t2 = 0.0, t3 = 0.0, t4 = 0.0;
#pragma unroll
      for (int p = 0; p < n1; ++p) {
        t1 += La_k[p * n1 + j] * c1[p];
        t2 += La_k[p * n1 + j] * c2[p];
        t3 += La_k[p * n1 + i] * c3[p];
        t4 += La_k[p * n1 + i] * c4[p];
      }
      acc[v] = z + lm1_i * t1 + lp1_i * t2 + lm1_j * t3 + lp1_j * t4;
    }
    const double* xv = sX + le * 16;
    const double minv = 1.0 / (pyr_jac(xv, ops.na[n], ops.nb[n]) * ops.wwc[n]);
    const double kap = mesh.mat[e * 4 + 0], irho = mesh.mat[e * 4 + 1];
    const double dte = dt * mesh.mat[e * 4 + 3];
    acc[0] -= source_term<Np>(mesh, e, n);
#pragma unroll
    for (int v = 0; v < 4; ++v)
      finish_coeff<MODE>(acc[v], minv, v == 0 ? kap : irho, out, R, (e * 4 + v) * Np + n, ra, rb,
                         dte);
  }
}

template <int N>
hipError_t trace_sf_n(const dgpyr_ctx& c, const double* U, double* T, hipStream_t s) {
  const int64_t nb = (c.K + SfDim<N>::E - 1) / SfDim<N>::E;
  hipLaunchKernelGGL(k_trace_sf<N>, dim3((unsigned)nb), dim3(kThreads), 0, s, U, T, c.sf, c.K);
  return hipGetLastError();
}

template <int N>
hipError_t stage_sf_n(const dgpyr_ctx& c, int mode, const double* U, const double* T, double* out,
                      double* R, double ra, double rb, double dt, hipStream_t s) {
  const int64_t nb = (c.K + SfDim<N>::E - 1) / SfDim<N>::E;
  if (mode == 0)
    hipLaunchKernelGGL((k_stage_sf<N, 0>), dim3((unsigned)nb), dim3(kThreads), 0, s, U, T, c.sf,
                       c.ops, c.mesh, out, R, ra, rb, dt);
  else
    hipLaunchKernelGGL((k_stage_sf<N, 1>), dim3((unsigned)nb), dim3(kThreads), 0, s, U, T, c.sf,
                       c.ops, c.mesh, out, R, ra, rb, dt);
  return hipGetLastError();
}

}  // namespace

#define DGPYR_DISPATCH_SF(fn, ...)        \
  switch (c.N) {                          \
    case 0: return fn<0>(__VA_ARGS__);    \
    case 1: return fn<1>(__VA_ARGS__);    \
    case 2: return fn<2>(__VA_ARGS__);    \
    case 3: return fn<3>(__VA_ARGS__);    \
    case 4: return fn<4>(__VA_ARGS__);    \
    case 5: return fn<5>(__VA_ARGS__);    \
    case 6: return fn<6>(__VA_ARGS__);    \
    case 7: return fn<7>(__VA_ARGS__);    \
    case 8: return fn<8>(__VA_ARGS__);    \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_trace_sf(const dgpyr_ctx& c, const double* U, double* T, hipStream_t s) {
  DGPYR_DISPATCH_SF(trace_sf_n, c, U, T, s)
}

hipError_t launch_stage_sf(const dgpyr_ctx& c, int mode, const double* U, const double* T,
                           double* out, double* R, double ra, double rb, double dt, hipStream_t s) {
  DGPYR_DISPATCH_SF(stage_sf_n, c, mode, U, T, out, R, ra, rb, dt, s)
}

}  // namespace dgpyr
