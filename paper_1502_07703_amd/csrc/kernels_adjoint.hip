// Transposed DG operator for the discrete adjoint.  With the semi-discrete
// system dU/dt = A U + b, A = -Kmat M^-1 D (Kmat = kappa on pressure rows,
// 1/rho on velocity rows; M diagonal, Lemma 3), the adjoint needs
//   A^T lam = -D^T mu,  mu = M^-1 Kmat lam.
// D = volume (strong form, Algorithm 1) + surface (Algorithm 2).
//   volume^T:  (D^T mu)_{u_k} = sum_rho D_rho^T W adj[rho][k] (V mu_p),
//              (D^T mu)_p     = sum_rho D_rho^T W sum_k adj[rho][k] (V mu_{u_k})
//   (one interpolation V mu, the pointwise metric, three projections with
//   D_rho^T: the forward contractions in reverse order, same flops);
//   surface^T: the flux is F = w sJ / 2 * G_n (U+ - U-) with G_n symmetric,
//              G_n = [[-tau_p, n^T], [n, -tau_u n n^T]]; its transpose at a
//              face point is g = w sJ / 2 * (G_{-n} mu'^f - G_n mu^f) with mu^f,
//              mu'^f the traces of mu on this and the neighbouring element
//              (on a boundary, g = w sJ / 2 * (B - I) G_n mu^f with the
//              mirror map B), lifted by (V^f)^T like the forward flux.
// FP64 matrix-core contractions, one 4-element group per wave.
#include <hip/hip_runtime.h>

#include "context.hpp"
#include "geom.hpp"
#include "mfma.hpp"

namespace dgpyr {
namespace {

constexpr int kWaves = 4;
constexpr int kEW = 4;
constexpr int kEB = kWaves * kEW;
constexpr int kBlock = 64 * kWaves;

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// mu = M^-1 Kmat lam, one thread per coefficient.
template <int N>
__global__ __launch_bounds__(256) void k_adjoint_scale(const double* __restrict__ lam,
                                                       double* __restrict__ mu, DevOps ops,
                                                       DevMesh mesh) {
  constexpr int Np = Tiles<N>::Np;
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= mesh.K * 4 * Np) return;
  const int64_t e = gid / (4 * Np);
  const int rem = (int)(gid - e * 4 * Np);
  const int f = rem / Np, i = rem - f * Np;
  double jc[4];
  pyr_jac_coeffs(mesh.verts + e * 16, jc);
  const double m = mesh.mat[e * 4 + (f == 0 ? 0 : 1)];
  mu[gid] = lam[gid] * m / (pyr_jac_eval(jc, ops.na[i], ops.nb[i]) * ops.wwc[i]);
}

// G_n v for G_n = [[-tp, n^T], [n, -tu n n^T]].
__device__ __forceinline__ void apply_g(const double n[3], double tp, double tu, const double v[4],
                                        double out[4]) {
  const double nu = n[0] * v[1] + n[1] * v[2] + n[2] * v[3];
  out[0] = -tp * v[0] + nu;
  const double s = v[0] - tu * nu;
  out[1] = n[0] * s;
  out[2] = n[1] * s;
  out[3] = n[2] * s;
}

// Transposed flux g at face point q of element e from the traces of mu (T).
template <int Nfq>
__device__ __forceinline__ void adjoint_flux(const double* __restrict__ T, const DevOps& ops,
                                             const DevMesh& mesh, const double* x, int64_t e,
                                             int q, double g[4]) {
  constexpr int Nfc = 5 * Nfq;
  const int f = q / Nfq, qq = q - f * Nfq;
  const double* tm = T + (e * Nfc + q) * 4;
  const double mm[4] = {tm[0], tm[1], tm[2], tm[3]};
  double Nv[3];
  pyr_face_normal(x, f, ops.fa[q], ops.fb[q], Nv);
  const double sJ = sqrt(Nv[0] * Nv[0] + Nv[1] * Nv[1] + Nv[2] * Nv[2]);
  const double n[3] = {Nv[0] / sJ, Nv[1] / sJ, Nv[2] / sJ};
  const double zm = mesh.mat[e * 4 + 2];
  const int nb = mesh.conn[e * 8 + f];
  const double hw = 0.5 * ops.wf[q] * sJ;
  double a[4];
  if (nb >= 0) {
    const int code = (mesh.conn[e * 8 + 5] >> (6 * f)) & 63;
    const int nf = code & 7, o = code >> 3;
    const int pi = ops.perm[(f == 0 ? o : 8 + o) * Nfq + qq];
    const double* tp = T + ((int64_t)nb * Nfc + nf * Nfq + pi) * 4;
    const double zp = mesh.mat[(int64_t)nb * 4 + 2];
    const double zavg = 0.5 * (zm + zp);
    const double taup = mesh.alpha / zavg, tauu = mesh.alpha * zavg;
    // G_{-n} mu' = D G_n D mu' with D = diag(1, -1, -1, -1)
    const double mp[4] = {tp[0], -tp[1], -tp[2], -tp[3]};
    double b[4];
    apply_g(n, taup, tauu, mp, b);
    apply_g(n, taup, tauu, mm, a);
    g[0] = hw * (b[0] - a[0]);
    g[1] = hw * (-b[1] - a[1]);
    g[2] = hw * (-b[2] - a[2]);
    g[3] = hw * (-b[3] - a[3]);
  } else {
    const double taup = mesh.alpha / zm, tauu = mesh.alpha * zm;
    apply_g(n, taup, tauu, mm, a);
    if (mesh.bc == DGPYR_BC_WALL) {  // B - I = [[0, 0], [0, -2 n n^T]]
      const double un = n[0] * a[1] + n[1] * a[2] + n[2] * a[3];
      g[0] = 0.0;
      g[1] = -2.0 * hw * un * n[0];
      g[2] = -2.0 * hw * un * n[1];
      g[3] = -2.0 * hw * un * n[2];
    } else {  // free surface: B - I = [[-2, 0], [0, 0]]
      g[0] = -2.0 * hw * a[0];
      g[1] = g[2] = g[3] = 0.0;
    }
  }
}

// out = A^T lam = -D^T mu; mu and its traces T precomputed.  A operands of
// mu: rows i = 4 f + e (FP64 layout, see mfma.hpp).
template <int N>
__global__ __launch_bounds__(kBlock, 2) void k_adjoint_mfma(const double* __restrict__ mu,
                                                            const double* __restrict__ T,
                                                            AdjOps ad, DevOps ops,
                                                            DevMesh mesh,
                                                            double* __restrict__ out) {
  using TT = Tiles<N>;
  using M = Mma<0>;
  constexpr int KP = Pack<double>::KP;
  constexpr int NCHP = (TT::NCH + KP - 1) / KP, NITP = (TT::NIT + KP - 1) / KP;
  __shared__ double sX[kEB][16];
  __shared__ double sQ[kWaves][16][17];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t eb0 = (int64_t)blockIdx.x * kEB;
  for (int x = threadIdx.x; x < kEB * 16; x += kBlock) {
    const int64_t e = eb0 + x / 16;
    sX[x / 16][x % 16] = e < mesh.K ? mesh.verts[e * 16 + (x % 16)] : 0.0;
  }
  const int64_t ew0 = eb0 + wv * kEW;
  const int row = lane & 15, kq = lane >> 4;
  double afr[TT::NCH];
  {
    const int64_t ea = ew0 + M::row_elem(row);
    const int f = M::row_field(row);
#pragma unroll
    for (int c = 0; c < TT::NCH; ++c) {
      const int n = 4 * c + kq;
      afr[c] = (ea < mesh.K && n < TT::Np) ? mu[(ea * 4 + f) * TT::Np + n] : 0.0;
    }
  }
  __syncthreads();
  const double* VrF = ad.VrF + lane * KP;
  const double* DrP = ad.DrP + lane * KP;
  const double* DsP = ad.DsP + lane * KP;
  const double* DtP = ad.DtP + lane * KP;
  const double* LfF = ad.LfP + lane * KP;
  const int de = lane >> 4, dq = lane & 15;
  const int64_t e = ew0 + de;
  const double* xv = sX[wv * kEW + de];
  M::Acc z[TT::NIT];
#pragma unroll
  for (int u = 0; u < TT::NIT; ++u) z[u] = M::zero();

  // volume^T: interpolate, metric, three projections
  for (int t = 0; t < TT::NTC; ++t) {
    M::Acc y = M::zero();
    const size_t fb = (size_t)t * NCHP * 64 * KP;
    dx2 pv;
#pragma unroll
    for (int c = 0; c < TT::NCH; ++c) {
      if (c % KP == 0) pv = load_pack(VrF + fb + (size_t)(c / KP) * 64 * KP);
      y = M::mma(afr[c], pv[c % KP], y);
    }
    const int q = 16 * t + dq;
    double Q[3][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    if (q < TT::Nc) {
      const int pm = q % TT::Nfq;
      double adj[9], J;
      pyr_metric(xv, ops.xg[pm % TT::n1], ops.xg[pm / TT::n1], adj, &J);
      const double w = ops.wv[q];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        Q[r][0] = w * (adj[3 * r] * y[1] + adj[3 * r + 1] * y[2] + adj[3 * r + 2] * y[3]);
#pragma unroll
        for (int k = 0; k < 3; ++k) Q[r][1 + k] = w * adj[3 * r + k] * y[0];
      }
    }
    const size_t pb = (size_t)t * 4 * NITP * 64 * KP;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const double* DP = r == 0 ? DrP : r == 1 ? DsP : DtP;
#pragma unroll
      for (int v = 0; v < 4; ++v) sQ[wv][M::row(de, v)][dq] = Q[r][v];
      wave_lds_sync();
#pragma unroll
      for (int c2 = 0; c2 < 4; ++c2) {
        const double a = sQ[wv][row][4 * c2 + kq];
        dx2 pk;
#pragma unroll
        for (int u = 0; u < TT::NIT; ++u) {
          if (u % KP == 0) pk = load_pack(DP + pb + ((size_t)c2 * NITP + u / KP) * 64 * KP);
          z[u] = M::mma(a, pk[u % KP], z[u]);
        }
      }
      wave_lds_sync();
    }
  }

  // surface^T: transposed flux at the face points, lifted by (V^f)^T
  for (int t = 0; t < TT::NTF; ++t) {
    const int q = 16 * t + dq;
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    if (e < mesh.K && q < TT::Nfc) adjoint_flux<TT::Nfq>(T, ops, mesh, xv, e, q, g);
#pragma unroll
    for (int v = 0; v < 4; ++v) sQ[wv][M::row(de, v)][dq] = g[v];
    wave_lds_sync();
    const size_t pb = (size_t)t * 4 * NITP * 64 * KP;
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) {
      const double a = sQ[wv][row][4 * c2 + kq];
      dx2 pk;
#pragma unroll
      for (int u = 0; u < TT::NIT; ++u) {
        if (u % KP == 0) pk = load_pack(LfF + pb + ((size_t)c2 * NITP + u / KP) * 64 * KP);
        z[u] = M::mma(a, pk[u % KP], z[u]);
      }
    }
    wave_lds_sync();
  }

  if (e >= mesh.K) return;
#pragma unroll
  for (int u = 0; u < TT::NIT; ++u) {
    const int i = 16 * u + dq;
    if (i >= TT::Np) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(e * 4 + v) * TT::Np + i] = -z[u][v];
  }
}

// Pressure at receivers: out[r] = sum_i phi_r[i] U[e_r][p][i].
__global__ void k_rec_sample(const double* __restrict__ U, const int64_t* __restrict__ elem,
                             const double* __restrict__ phi, int nrec, int Np,
                             double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrec) return;
  const double* u = U + elem[r] * 4 * Np;
  const double* f = phi + (int64_t)r * Np;
  double acc = 0.0;
  for (int i = 0; i < Np; ++i) acc += f[i] * u[i];
  out[r] = acc;
}

// Ubar[e_r][p][i] += coef[r] phi_r[i]; thread i walks the receivers in order,
// so receivers sharing an element add without races.
__global__ void k_rec_inject(double* __restrict__ Ub, const int64_t* __restrict__ elem,
                             const double* __restrict__ phi, const double* __restrict__ coef,
                             int nrec, int Np) {
  const int i = threadIdx.x;
  if (i >= Np) return;
  for (int r = 0; r < nrec; ++r) Ub[elem[r] * 4 * Np + i] += coef[r] * phi[(int64_t)r * Np + i];
}

// Reverse LSRK stage, before the transposed operator: Rb += b_s Ub.
__global__ void k_adj_pre(double* __restrict__ Rb, const double* __restrict__ Ub, double bs,
                          int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) Rb[i] += bs * Ub[i];
}

// After it: Ub += dt (A^T Rb), then Rb *= a_s.
__global__ void k_adj_post(double* __restrict__ Ub, double* __restrict__ Rb,
                           const double* __restrict__ ATRb, double dt, double as, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    Ub[i] += dt * ATRb[i];
    Rb[i] *= as;
  }
}

// grad[e] += dt sum_i Rb[e][p][i] F[e][p][i] / kappa_e (F: the stage's
// right-hand side; its pressure rows carry the factor kappa_e).
__global__ void k_kappa_grad(double* __restrict__ grad, const double* __restrict__ Rb,
                             const double* __restrict__ F, const double* __restrict__ mat,
                             int64_t K, int Np, double dt) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= K) return;
  const double* r = Rb + e * 4 * Np;
  const double* f = F + e * 4 * Np;
  double acc = 0.0;
  for (int i = 0; i < Np; ++i) acc += r[i] * f[i];
  grad[e] += dt * acc / mat[e * 4];
}

// kappa derivative through the penalty coefficients (alpha > 0, Section 4.3):
// tau_p = alpha/{rho c}, tau_u = alpha {rho c}, {rho c} = (z- + z+)/2,
// z = sqrt(kappa rho).  At a face point of element e, with jumps of the
// forward state W (traces TW) and mu = M^-1 Kmat Rb (traces TM),
//   s_e = -w sJ alpha/2 (mu_p [[p]] / {rho c}^2 - (n.mu_u)(n.[[u]]))
// is d/d{rho c} of <Rb_e, (A W)_e> there.  Element K collects, over its face
// points, s_K and the neighbour's s at the matching point (the same {rho c}
// enters the neighbour's rows), times d{rho c}/d kappa_K = z_K / (4 kappa_K);
// a boundary face (ghost with the element's material) gives
// s_K z_K / (2 kappa_K).  One wave per element, its lanes over the face
// points, summed in a fixed order through LDS (deterministic, no atomics).
constexpr int kTauWaves = 4;
__global__ __launch_bounds__(64 * kTauWaves) void k_tau_grad(
    double* __restrict__ grad, const double* __restrict__ TW, const double* __restrict__ TM,
    DevOps ops, DevMesh mesh, int Nfq, double dt) {
  __shared__ double sAcc[64 * kTauWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * kTauWaves + wv;
  const int Nfc = 5 * Nfq;
  double acc = 0.0;
  if (e < mesh.K) {
    const double* x = mesh.verts + e * 16;
    const double kap = mesh.mat[e * 4 + 0], z = mesh.mat[e * 4 + 2];
    for (int q = lane; q < Nfc; q += 64) {
      const int f = q / Nfq, qq = q - f * Nfq;
      const double* tm = TW + (e * Nfc + q) * 4;
      const double* mm = TM + (e * Nfc + q) * 4;
      double Nv[3];
      pyr_face_normal(x, f, ops.fa[q], ops.fb[q], Nv);
      const double sJ = sqrt(Nv[0] * Nv[0] + Nv[1] * Nv[1] + Nv[2] * Nv[2]);
      const double n0 = Nv[0] / sJ, n1 = Nv[1] / sJ, n2 = Nv[2] / sJ;
      const double c = -0.5 * ops.wf[q] * sJ * mesh.alpha;
      const double mun = n0 * mm[1] + n1 * mm[2] + n2 * mm[3];
      const int nb = mesh.conn[e * 8 + f];
      if (nb >= 0) {
        const int code = (mesh.conn[e * 8 + 5] >> (6 * f)) & 63;
        const int nf = code & 7, o = code >> 3;
        const int pi = ops.perm[(f == 0 ? o : 8 + o) * Nfq + qq];
        const double* tp = TW + ((int64_t)nb * Nfc + nf * Nfq + pi) * 4;
        const double* mp = TM + ((int64_t)nb * Nfc + nf * Nfq + pi) * 4;
        const double jp = tp[0] - tm[0];
        const double jun = n0 * (tp[1] - tm[1]) + n1 * (tp[2] - tm[2]) + n2 * (tp[3] - tm[3]);
        const double zavg = 0.5 * (z + mesh.mat[(int64_t)nb * 4 + 2]);
        const double iz2 = 1.0 / (zavg * zavg);
        const double s_own = c * (mm[0] * jp * iz2 - mun * jun);
        const double mpn = n0 * mp[1] + n1 * mp[2] + n2 * mp[3];
        const double s_nb = c * (-mp[0] * jp * iz2 + mpn * jun);
        acc += (s_own + s_nb) * z / (4.0 * kap);
      } else {
        double jp, jun;
        if (mesh.bc == DGPYR_BC_WALL) {
          jp = 0.0;
          jun = -2.0 * (n0 * tm[1] + n1 * tm[2] + n2 * tm[3]);
        } else {
          jp = -2.0 * tm[0];
          jun = 0.0;
        }
        const double s_own = c * (mm[0] * jp / (z * z) - mun * jun);
        acc += s_own * z / (2.0 * kap);
      }
    }
  }
  sAcc[threadIdx.x] = acc;
  __syncthreads();
  if (lane == 0 && e < mesh.K) {
    double sum = 0.0;
    for (int l = 0; l < 64; ++l) sum += sAcc[wv * 64 + l];
    grad[e] += dt * sum;
  }
}

template <int N>
hipError_t adjoint_n(const dgpyr_ctx& c, const double* mu, const double* T, double* out,
                     hipStream_t s) {
  const int64_t nb = (c.K + kEB - 1) / kEB;
  hipLaunchKernelGGL((k_adjoint_mfma<N>), dim3((unsigned)nb), dim3(kBlock), 0, s, mu, T, c.adj,
                     c.ops, c.mesh, out);
  return hipGetLastError();
}

template <int N>
hipError_t adjoint_scale_n(const dgpyr_ctx& c, const double* lam, double* mu, hipStream_t s) {
  const int64_t n = c.K * 4 * c.Np;
  hipLaunchKernelGGL((k_adjoint_scale<N>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, lam,
                     mu, c.ops, c.mesh);
  return hipGetLastError();
}

}  // namespace

#define DGPYR_DISPATCH_ADJ(fn, ...)       \
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

hipError_t launch_adjoint_scale(const dgpyr_ctx& c, const double* lam, double* mu, hipStream_t s) {
  DGPYR_DISPATCH_ADJ(adjoint_scale_n, c, lam, mu, s)
}

hipError_t launch_adjoint(const dgpyr_ctx& c, const double* mu, const double* T, double* out,
                          hipStream_t s) {
  DGPYR_DISPATCH_ADJ(adjoint_n, c, mu, T, out, s)
}

static inline unsigned blocks256(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_rec_sample(const dgpyr_ctx& c, const double* U, double* out, hipStream_t s) {
  if (c.nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rec_sample, dim3(blocks256(c.nrec)), dim3(256), 0, s, U, c.rec_elem,
                     c.rec_phi, c.nrec, c.Np, out);
  return hipGetLastError();
}

hipError_t launch_rec_inject(const dgpyr_ctx& c, double* Ub, const double* coef, hipStream_t s) {
  if (c.nrec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rec_inject, dim3(1), dim3(256), 0, s, Ub, c.rec_elem, c.rec_phi, coef,
                     c.nrec, c.Np);
  return hipGetLastError();
}

hipError_t launch_adj_pre(const dgpyr_ctx& c, double* Rb, const double* Ub, double bs,
                          hipStream_t s) {
  const int64_t n = c.K * 4 * c.Np;
  hipLaunchKernelGGL(k_adj_pre, dim3(blocks256(n)), dim3(256), 0, s, Rb, Ub, bs, n);
  return hipGetLastError();
}

hipError_t launch_adj_post(const dgpyr_ctx& c, double* Ub, double* Rb, const double* ATRb,
                           double dt, double as, hipStream_t s) {
  const int64_t n = c.K * 4 * c.Np;
  hipLaunchKernelGGL(k_adj_post, dim3(blocks256(n)), dim3(256), 0, s, Ub, Rb, ATRb, dt, as, n);
  return hipGetLastError();
}

hipError_t launch_tau_grad(const dgpyr_ctx& c, double* grad, const double* TW, const double* TM,
                           double dt, hipStream_t s) {
  const int64_t nb = (c.K + kTauWaves - 1) / kTauWaves;
  hipLaunchKernelGGL(k_tau_grad, dim3((unsigned)nb), dim3(64 * kTauWaves), 0, s, grad, TW, TM,
                     c.ops, c.mesh, c.Nfq, dt);
  return hipGetLastError();
}

hipError_t launch_kappa_grad(const dgpyr_ctx& c, double* grad, const double* Rb, const double* F,
                             double dt, hipStream_t s) {
  hipLaunchKernelGGL(k_kappa_grad, dim3(blocks256(c.K)), dim3(256), 0, s, grad, Rb, F,
                     c.mesh.mat, c.K, c.Np, dt);
  return hipGetLastError();
}

}  // namespace dgpyr
