// Reference FP64 kernels: trace interpolation, volume term, surface term with
// inverse mass and LSRK update (Algorithms 1-3).  One workgroup owns E
// consecutive elements and stages their coefficients in LDS; operators are read
// from global memory in layouts where consecutive lanes touch consecutive
// addresses.
#include <hip/hip_runtime.h>

#include "context.hpp"
#include "flux.hpp"
#include "geom.hpp"

namespace dgpyr {
namespace {

constexpr int kThreads = 256;

template <int N>
struct Dim {
  static constexpr int n1 = N + 1;
  static constexpr int Np = (N + 1) * (N + 2) * (2 * N + 3) / 6;
  static constexpr int Nc = n1 * n1 * n1;
  static constexpr int Nfq = n1 * n1;
  static constexpr int Nfc = 5 * Nfq;
  // elements per workgroup; keeps static LDS under 64 KiB for every N
  static constexpr int E = N <= 1 ? 16 : N <= 3 ? 8 : N <= 5 ? 4 : N <= 6 ? 2 : 1;
};

// U in the canonical layout [K][4][Np]; T in [K][Nfc][4].
template <int N>
__global__ __launch_bounds__(kThreads) void k_trace(const double* __restrict__ U,
                                                    double* __restrict__ T, DevOps ops, int64_t K) {
  using D = Dim<N>;
  __shared__ double sU[D::E * 4 * D::Np];
  const int64_t e0 = (int64_t)blockIdx.x * D::E;
  const int ne = (int)((K - e0) < D::E ? (K - e0) : D::E);
  const double* Ub = U + e0 * 4 * D::Np;
  for (int x = threadIdx.x; x < ne * 4 * D::Np; x += kThreads) sU[x] = Ub[x];
  __syncthreads();
  for (int x = threadIdx.x; x < ne * D::Nfc; x += kThreads) {
    const int le = x / D::Nfc, q = x - le * D::Nfc;
    const double* su = sU + le * 4 * D::Np;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int n = 0; n < D::Np; ++n) {
      const double v = ops.VfT[n * D::Nfc + q];
      a0 += v * su[n];
      a1 += v * su[D::Np + n];
      a2 += v * su[2 * D::Np + n];
      a3 += v * su[3 * D::Np + n];
    }
    double* o = T + ((e0 + le) * D::Nfc + q) * 4;
    o[0] = a0; o[1] = a1; o[2] = a2; o[3] = a3;
  }
}

// Volume term (Algorithm 1, strong form): at each cubature point the twelve
// reference derivatives d_rho u_f, then with adj = J dR/dx (constant along c)
//   Q_p   = w sum_rho sum_k adj[rho][k] d_rho u_k    (= w J div u)
//   Q_u_k = w sum_rho adj[rho][k] d_rho p            (= w J dp/dx_k)
// and vol_f,i = sum_q phi_i(q) Q_f(q).
template <int N>
__global__ __launch_bounds__(kThreads) void k_volume(const double* __restrict__ U,
                                                     double* __restrict__ vol, DevOps ops,
                                                     DevMesh mesh) {
  using D = Dim<N>;
  __shared__ double sU[D::E * 4 * D::Np];
  __shared__ double sQ[D::E * 4 * D::Nc];
  __shared__ double sX[D::E * 16];
  const int64_t e0 = (int64_t)blockIdx.x * D::E;
  const int ne = (int)((mesh.K - e0) < D::E ? (mesh.K - e0) : D::E);
  const double* Ub = U + e0 * 4 * D::Np;
  for (int x = threadIdx.x; x < ne * 4 * D::Np; x += kThreads) sU[x] = Ub[x];
  for (int x = threadIdx.x; x < ne * 16; x += kThreads) sX[x] = mesh.verts[e0 * 16 + x];
  __syncthreads();
  for (int x = threadIdx.x; x < ne * D::Nc; x += kThreads) {
    const int le = x / D::Nc, q = x - le * D::Nc;
    const int p = q % D::n1, m = (q / D::n1) % D::n1;
    const double* su = sU + le * 4 * D::Np;
    double d[3][4] = {};
    for (int n = 0; n < D::Np; ++n) {
      const double dr = ops.DrT[n * D::Nc + q];
      const double ds = ops.DsT[n * D::Nc + q];
      const double dt = ops.DtT[n * D::Nc + q];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const double u = su[f * D::Np + n];
        d[0][f] += dr * u;
        d[1][f] += ds * u;
        d[2][f] += dt * u;
      }
    }
    double adj[9], J;
    pyr_metric(sX + le * 16, ops.xg[p], ops.xg[m], adj, &J);
    const double w = ops.wv[q];
    double qp = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) qp += adj[3 * r + k] * d[r][1 + k];
    double* sq = sQ + le * 4 * D::Nc;
    sq[q] = w * qp;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      sq[(1 + k) * D::Nc + q] = w * (adj[k] * d[0][0] + adj[3 + k] * d[1][0] + adj[6 + k] * d[2][0]);
  }
  __syncthreads();
  for (int x = threadIdx.x; x < ne * D::Np; x += kThreads) {
    const int le = x / D::Np, i = x - le * D::Np;
    const double* sq = sQ + le * 4 * D::Nc;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (int q = 0; q < D::Nc; ++q) {
      const double v = ops.V[q * D::Np + i];
      a0 += v * sq[q];
      a1 += v * sq[D::Nc + q];
      a2 += v * sq[2 * D::Nc + q];
      a3 += v * sq[3 * D::Nc + q];
    }
    double* o = vol + (e0 + le) * 4 * D::Np;
    o[i] = a0;
    o[D::Np + i] = a1;
    o[2 * D::Np + i] = a2;
    o[3 * D::Np + i] = a3;
  }
}

// Surface term (Algorithm 2), inverse mass and material scaling, and the LSRK
// update (Algorithm 3).  With jumps [[q]] = q+ - q- and outward unit normal n:
//   P_p = (n.[[u]] - tau_p [[p]]) / 2,  P_u = ([[p]] - tau_u n.[[u]]) / 2,
//   F_p = w sJ P_p,  F_u_k = w sJ n_k P_u,   lift_f,i = sum_q phi_i(q) F_f(q);
//   rhs_p = -kappa (vol + lift)_p / M_ii,  rhs_u = -(1/rho) (vol + lift)_u / M_ii,
//   M_ii = J(a_i, b_i) w_i^k w_j^k 2/(2k+3)  (Lemma 3).
template <int N, int MODE>
__global__ __launch_bounds__(kThreads) void k_surface(const double* __restrict__ T,
                                                      const double* __restrict__ vol, DevOps ops,
                                                      DevMesh mesh, double* out, double* R,
                                                      double ra, double rb, double dt) {
  using D = Dim<N>;
  __shared__ double sF[D::E * 4 * D::Nfc];
  __shared__ double sX[D::E * 16];
  const int64_t e0 = (int64_t)blockIdx.x * D::E;
  const int ne = (int)((mesh.K - e0) < D::E ? (mesh.K - e0) : D::E);
  for (int x = threadIdx.x; x < ne * 16; x += kThreads) sX[x] = mesh.verts[e0 * 16 + x];
  __syncthreads();
  for (int x = threadIdx.x; x < ne * D::Nfc; x += kThreads) {
    const int le = x / D::Nfc, q = x - le * D::Nfc;
    const int f = q / D::Nfq, qq = q - f * D::Nfq;
    const int64_t e = e0 + le;
    const double* tm = T + (e * D::Nfc + q) * 4;
    const double pm = tm[0], um0 = tm[1], um1 = tm[2], um2 = tm[3];
    double Nv[3];
    pyr_face_normal(sX + le * 16, f, ops.fa[q], ops.fb[q], Nv);
    const double sJ = sqrt(Nv[0] * Nv[0] + Nv[1] * Nv[1] + Nv[2] * Nv[2]);
    const double n0 = Nv[0] / sJ, n1 = Nv[1] / sJ, n2 = Nv[2] / sJ;
    const double zm = mesh.mat[e * 4 + 2];
    const int nb = mesh.conn[e * 8 + f];
    double pp, up0, up1, up2, zp;
    if (nb >= 0) {
      const int code = (mesh.conn[e * 8 + 5] >> (6 * f)) & 63;
      const int nf = code & 7, o = code >> 3;
      const int pi = ops.perm[(f == 0 ? o : 8 + o) * D::Nfq + qq];
      const double* tp = T + ((int64_t)nb * D::Nfc + nf * D::Nfq + pi) * 4;
      pp = tp[0]; up0 = tp[1]; up1 = tp[2]; up2 = tp[3];
      zp = mesh.mat[(int64_t)nb * 4 + 2];
    } else {
      const double un = n0 * um0 + n1 * um1 + n2 * um2;
      if (mesh.bc == DGPYR_BC_WALL) {
        pp = pm; up0 = um0 - 2 * un * n0; up1 = um1 - 2 * un * n1; up2 = um2 - 2 * un * n2;
      } else {
        pp = -pm; up0 = um0; up1 = um1; up2 = um2;
      }
      zp = zm;
    }
    const double zavg = 0.5 * (zm + zp);
    const double taup = mesh.alpha / zavg, tauu = mesh.alpha * zavg;
    const double jp = pp - pm;
    const double jun = n0 * (up0 - um0) + n1 * (up1 - um1) + n2 * (up2 - um2);
    const double w = ops.wf[q] * sJ;
    const double Pp = 0.5 * w * (jun - taup * jp);
    const double Pu = 0.5 * w * (jp - tauu * jun);
    double* sf = sF + le * 4 * D::Nfc;
    sf[q] = Pp;
    sf[D::Nfc + q] = n0 * Pu;
    sf[2 * D::Nfc + q] = n1 * Pu;
    sf[3 * D::Nfc + q] = n2 * Pu;
  }
  __syncthreads();
  for (int x = threadIdx.x; x < ne * D::Np; x += kThreads) {
    const int le = x / D::Np, i = x - le * D::Np;
    const int64_t e = e0 + le;
    const double* sf = sF + le * 4 * D::Nfc;
    const double* vo = vol + e * 4 * D::Np;
    double acc[4] = {vo[i], vo[D::Np + i], vo[2 * D::Np + i], vo[3 * D::Np + i]};
    for (int q = 0; q < D::Nfc; ++q) {
      const double v = ops.Vf[q * D::Np + i];
#pragma unroll
      for (int f = 0; f < 4; ++f) acc[f] += v * sf[f * D::Nfc + q];
    }
    const double J = pyr_jac(sX + le * 16, ops.na[i], ops.nb[i]);
    const double minv = 1.0 / (J * ops.wwc[i]);
    const double kap = mesh.mat[e * 4 + 0], irho = mesh.mat[e * 4 + 1];
    const double dte = dt * mesh.mat[e * 4 + 3];
    acc[0] -= source_term<D::Np>(mesh, e, i);
    double rhs[4];
    rhs[0] = -kap * minv * acc[0];
#pragma unroll
    for (int f = 1; f < 4; ++f) rhs[f] = -irho * minv * acc[f];
    double* o = out + e * 4 * D::Np;
    if (MODE == 0) {
#pragma unroll
      for (int f = 0; f < 4; ++f) o[f * D::Np + i] = rhs[f];
    } else {
      double* r = R + e * 4 * D::Np;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const double rn = (ra == 0.0 ? 0.0 : ra * r[f * D::Np + i]) + dte * rhs[f];
        r[f * D::Np + i] = rn;
        o[f * D::Np + i] += rb * rn;
      }
    }
  }
}

template <int N>
hipError_t trace_n(const dgpyr_ctx& c, const double* U, double* T, hipStream_t s) {
  const int64_t nb = (c.K + Dim<N>::E - 1) / Dim<N>::E;
  hipLaunchKernelGGL(k_trace<N>, dim3((unsigned)nb), dim3(kThreads), 0, s, U, T, c.ops, c.K);
  return hipGetLastError();
}

template <int N>
hipError_t volume_n(const dgpyr_ctx& c, const double* U, double* vol, hipStream_t s) {
  const int64_t nb = (c.K + Dim<N>::E - 1) / Dim<N>::E;
  hipLaunchKernelGGL(k_volume<N>, dim3((unsigned)nb), dim3(kThreads), 0, s, U, vol, c.ops, c.mesh);
  return hipGetLastError();
}

template <int N>
hipError_t surface_n(const dgpyr_ctx& c, int mode, const double* T, const double* vol, double* out,
                     double* R, double ra, double rb, double dt, hipStream_t s) {
  const int64_t nb = (c.K + Dim<N>::E - 1) / Dim<N>::E;
  if (mode == 0)
    hipLaunchKernelGGL((k_surface<N, 0>), dim3((unsigned)nb), dim3(kThreads), 0, s, T, vol, c.ops,
                       c.mesh, out, R, ra, rb, dt);
  else
    hipLaunchKernelGGL((k_surface<N, 1>), dim3((unsigned)nb), dim3(kThreads), 0, s, T, vol, c.ops,
                       c.mesh, out, R, ra, rb, dt);
  return hipGetLastError();
}

}  // namespace

#define DGPYR_DISPATCH(fn, ...)                 \
  switch (c.N) {                                \
    case 0: return fn<0>(__VA_ARGS__);          \
    case 1: return fn<1>(__VA_ARGS__);          \
    case 2: return fn<2>(__VA_ARGS__);          \
    case 3: return fn<3>(__VA_ARGS__);          \
    case 4: return fn<4>(__VA_ARGS__);          \
    case 5: return fn<5>(__VA_ARGS__);          \
    case 6: return fn<6>(__VA_ARGS__);          \
    case 7: return fn<7>(__VA_ARGS__);          \
    case 8: return fn<8>(__VA_ARGS__);          \
    default: return hipErrorInvalidValue;       \
  }

hipError_t launch_trace(const dgpyr_ctx& c, const double* U, double* T, hipStream_t s) {
  DGPYR_DISPATCH(trace_n, c, U, T, s)
}
hipError_t launch_volume(const dgpyr_ctx& c, const double* U, double* vol, hipStream_t s) {
  DGPYR_DISPATCH(volume_n, c, U, vol, s)
}
hipError_t launch_surface(const dgpyr_ctx& c, int mode, const double* T, const double* vol,
                          double* out, double* R, double ra, double rb, double dt, hipStream_t s) {
  DGPYR_DISPATCH(surface_n, c, mode, T, vol, out, R, ra, rb, dt, s)
}

}  // namespace dgpyr
