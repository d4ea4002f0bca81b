// Matrix-core kernels for linear advection u_t + div(beta u) = 0 (Section 4.1;
// Algorithms 1-3 are stated for this equation): the trace interpolation and
// one fused stage (volume, surface lift, inverse mass, LSRK update).
//
// One field per element, so the 16 rows of an FP64 16x16x4 MFMA tile are 16
// elements: a wave owns 16 elements, a workgroup of 4 waves owns 64.  Lane l
// holds the A operand A[l % 16][l / 16] (element l % 16) and ends with
// D[4 v + l / 16][l % 16], v = 0..3 (elements 4 v + l / 16 at column l % 16),
// the FP64 lane layout measured on gfx950.  The operator fragments are the
// acoustic path's FP64 fragments (the B operand does not depend on what the
// rows mean).
#include <hip/hip_runtime.h>

#include "context.hpp"
#include "flux.hpp"
#include "geom.hpp"
#include "mfma.hpp"

namespace dgpyr {
namespace {

constexpr int kWaves = 4;
constexpr int kEW = 16;             // elements per wave
constexpr int kEB = kWaves * kEW;   // elements per workgroup
constexpr int kBlock = 64 * kWaves;

// Orders this wave's LDS writes before its later LDS reads and reads before
// later writes: a wave's LDS operations complete in issue order, the fences
// keep the compiler from moving LDS accesses across this point.
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A operands of u for 16 elements from ew0: lane l holds u[ew0 + l%16][4c + l/16],
// zero beyond Np or beyond the mesh.
template <int N>
__device__ __forceinline__ void load_adv_frags(const double* U, int64_t ew0,
                                               int64_t K, int lane, double* afr) {
  using TT = Tiles<N>;
  const int row = lane & 15, kq = lane >> 4;
  const int64_t e = ew0 + row;
  const double* src = U + e * TT::Np;
#pragma unroll
  for (int c = 0; c < TT::NCH; ++c) {
    const int n = 4 * c + kq;
    afr[c] = (e < K && n < TT::Np) ? src[n] : 0.0;
  }
}

// Own and neighbour traces at one face point (up = 0 on a face without a
// partner).
struct AdvTraces {
  double um, up;
};

// Neighbour of one element face: element, offset of its matching face in its
// trace row, row of the face-point permutation table.
struct AdvNb {
  int nb, off, prow;
};

// Weighted face term at face point q (face f) of an element with vertices x:
// w sJ (beta_n - alpha |beta_n|) / 2 (u+ - u-), with beta_n sJ = beta . N for
// the area-weighted outward normal N (no square root needed).
__device__ __forceinline__ double adv_flux_from(const AdvTraces& t, const DevOps& ops,
                                                const AdvParams& ap, const double* x, int f,
                                                int q) {
  double Nv[3];
  pyr_face_normal(x, f, ops.fa[q], ops.fb[q], Nv);
  const double bN = ap.beta[0] * Nv[0] + ap.beta[1] * Nv[1] + ap.beta[2] * Nv[2];
  return 0.5 * ops.wf[q] * (bN - ap.alpha * fabs(bN)) * (t.up - t.um);
}

// Traces T[K][Nfc] = V^f u (Algorithm 3's interpolation to face points).  A
// wave owns G groups of 16 elements; each operator fragment loaded feeds G
// products.
template <int N, int G>
__global__ __launch_bounds__(kBlock) void k_adv_trace(const double* __restrict__ U,
                                                      double* __restrict__ T, FragOps fo,
                                                      int64_t K) {
  using TT = Tiles<N>;
  using M = Mma<0>;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t ew0 = (int64_t)blockIdx.x * (kEB * G) + wv * (kEW * G);
  double afr[G][TT::NCH];
#pragma unroll
  for (int g = 0; g < G; ++g) load_adv_frags<N>(U, ew0 + kEW * g, K, lane, afr[g]);
  constexpr int KP = Pack<double>::KP;
  constexpr int NCHP = (TT::NCH + KP - 1) / KP;
  const double* VfF = static_cast<const double*>(fo.VfF) + lane * KP;
  const int de = lane >> 4, dq = lane & 15;
  for (int t = 0; t < TT::NTF; ++t) {
    M::Acc y[G];
#pragma unroll
    for (int g = 0; g < G; ++g) y[g] = M::zero();
    const size_t fb = (size_t)t * NCHP * 64 * KP;
    dx2 pk;
#pragma unroll
    for (int c = 0; c < TT::NCH; ++c) {
      if (c % KP == 0) pk = load_pack(VfF + fb + (size_t)(c / KP) * 64 * KP);
#pragma unroll
      for (int g = 0; g < G; ++g) y[g] = M::mma(afr[g][c], pk[c % KP], y[g]);
    }
    const int q = 16 * t + dq;
    if (q >= TT::Nfc) continue;
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t e = ew0 + kEW * g + 4 * v + de;
        if (e < K) T[e * TT::Nfc + q] = y[g][v];
      }
  }
}

// Waves per SIMD the stage kernel is compiled for (register budget 512 /
// waves).  Up to N = 6 the kernel fits without spilling; N = 7 and 8 spill
// at two waves (50 and 244 registers, with the surface loop left rolled) and
// are still faster than at one: 17.2 -> 13.9 ms and 35.2 -> 30.5 ms at
// 40^3 x 6 periodic pyramids.
template <int N>
struct AdvWaves {
  static constexpr int value = N <= 4 ? 3 : 2;
};

// Fused stage.  Volume (Algorithm 1): Y_rho = D_rho u at 16 cubature points
// per tile, then Q = w (beta . adj_r Y_r + beta . adj_s Y_s + beta . adj_t Y_t)
// with adj = J d(r, s, t)/dx from the element's vertices at the point's (a, b)
// (constant along c), then S u += V^T Q.  Surface (Algorithm 2): the face term
// at 16 face points per tile, lifted by V^f^T.  Then (Algorithm 3) the
// diagonal inverse mass 1 / (J(a_i, b_i) w_i w_j 2/(2k+3)) and the LSRK
// stage, du/dt = -M^-1 (S u + L^f F).  The workgroup reads and writes only its
// own elements' u and R; neighbours' values come from T, so the in-place
// update is safe.
template <int N, int MODE>
__global__ __launch_bounds__(kBlock, AdvWaves<N>::value) void k_adv_stage(
    const double* U, const double* __restrict__ T, FragOps fo, DevOps ops,
    DevMesh mesh, AdvParams ap, double* out, double* R, double ra, double rb, double dt) {
  using TT = Tiles<N>;
  using M = Mma<0>;
  __shared__ double sX[kEB][16];
  __shared__ double sQ[kWaves][16][17];
  __shared__ AdvNb sNb[kEB][5];
  __shared__ int sPerm[10 * TT::Nfq];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t eb0 = (int64_t)blockIdx.x * kEB;
  for (int x = threadIdx.x; x < kEB * 16; x += kBlock) {
    const int64_t e = eb0 + x / 16;
    sX[x / 16][x % 16] = e < mesh.K ? mesh.verts[e * 16 + (x % 16)] : 0.0;
  }
  for (int x = threadIdx.x; x < kEB * 5; x += kBlock) {
    const int le = x / 5, f = x - le * 5;
    const int64_t e = eb0 + le;
    AdvNb fn{-1, 0, 0};
    if (e < mesh.K) {
      const int nb = mesh.conn[e * 8 + f];
      if (nb >= 0) {
        const int code = (mesh.conn[e * 8 + 5] >> (6 * f)) & 63;
        const int nf = code & 7, o = code >> 3;
        fn = AdvNb{nb, nf * TT::Nfq, (f == 0 ? o : 8 + o) * TT::Nfq};
      }
    }
    sNb[le][f] = fn;
  }
  for (int x = threadIdx.x; x < 10 * TT::Nfq; x += kBlock) sPerm[x] = ops.perm[x];
  const int64_t ew0 = eb0 + wv * kEW;
  double afr[TT::NCH];
  load_adv_frags<N>(U, ew0, mesh.K, lane, afr);
  __syncthreads();

  constexpr int KP = Pack<double>::KP;
  constexpr int NCHP = (TT::NCH + KP - 1) / KP, NITP = (TT::NIT + KP - 1) / KP;
  const double* DrF = static_cast<const double*>(fo.DrF) + lane * KP;
  const double* DsF = static_cast<const double*>(fo.DsF) + lane * KP;
  const double* DtF = static_cast<const double*>(fo.DtF) + lane * KP;
  const double* VF = static_cast<const double*>(fo.VF) + lane * KP;
  const double* LfF = static_cast<const double*>(fo.LfF) + lane * KP;
  const int de = lane >> 4, dq = lane & 15;
  const int row = lane & 15, kq = lane >> 4;
  M::Acc z[TT::NIT];
#pragma unroll
  for (int u = 0; u < TT::NIT; ++u) z[u] = M::zero();

  // volume
  for (int t = 0; t < TT::NTC; ++t) {
    M::Acc yr = M::zero(), ys = M::zero(), yt = M::zero();
    const size_t fb = (size_t)t * NCHP * 64 * KP;
    dx2 pr, ps, pt;
#pragma unroll
    for (int c = 0; c < TT::NCH; ++c) {
      if (c % KP == 0) {
        const size_t o = fb + (size_t)(c / KP) * 64 * KP;
        pr = load_pack(DrF + o);
        ps = load_pack(DsF + o);
        pt = load_pack(DtF + o);
      }
      yr = M::mma(afr[c], pr[c % KP], yr);
      ys = M::mma(afr[c], ps[c % KP], ys);
      yt = M::mma(afr[c], pt[c % KP], yt);
      // at most a few chunks of operand loads in flight (registers)
      if ((c & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    const int q = 16 * t + dq;
    const int pm = q % TT::Nfq;
    const double a = ops.xg[pm % TT::n1], b = ops.xg[pm / TT::n1];
    const double w = q < TT::Nc ? ops.wv[q] : 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int le = 4 * v + de;
      double Q = 0.0;
      if (q < TT::Nc) {
        double adj[9], J;
        pyr_metric(sX[wv * kEW + le], a, b, adj, &J);
        const double br = ap.beta[0] * adj[0] + ap.beta[1] * adj[1] + ap.beta[2] * adj[2];
        const double bs = ap.beta[0] * adj[3] + ap.beta[1] * adj[4] + ap.beta[2] * adj[5];
        const double bt = ap.beta[0] * adj[6] + ap.beta[1] * adj[7] + ap.beta[2] * adj[8];
        Q = w * (br * yr[v] + bs * ys[v] + bt * yt[v]);
      }
      sQ[wv][le][dq] = Q;
    }
    wave_sync_lds();
    const size_t pb = (size_t)t * 4 * NITP * 64 * KP;
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) {
      const double av = sQ[wv][row][4 * c2 + kq];
      dx2 pv;
#pragma unroll
      for (int u = 0; u < TT::NIT; ++u) {
        if (u % KP == 0) pv = load_pack(VF + pb + ((size_t)c2 * NITP + u / KP) * 64 * KP);
        z[u] = M::mma(av, pv[u % KP], z[u]);
      }
    }
    wave_sync_lds();
  }

  // surface: the traces of tile t + 1 are gathered while tile t's face terms
  // and lift run.
  auto gather = [&](int v, int q, AdvTraces& tr) {
    const int le = 4 * v + de;
    const int64_t e = ew0 + le;
    const int f = q / TT::Nfq, qq = q - f * TT::Nfq;
    tr.um = T[e * TT::Nfc + q];
    const AdvNb& fn = sNb[wv * kEW + le][f];
    tr.up = fn.nb >= 0 ? T[(int64_t)fn.nb * TT::Nfc + fn.off + sPerm[fn.prow + qq]] : 0.0;
  };
  // unrolled up to N = 6; above, the unrolled loop needs some 230 more
  // registers than two waves per SIMD allow
  constexpr int kSurfUnroll = N <= 6 ? TT::NTF : 1;
  AdvTraces cur[4];
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (ew0 + 4 * v + de < mesh.K && dq < TT::Nfc) gather(v, dq, cur[v]);
#pragma unroll kSurfUnroll
  for (int t = 0; t < TT::NTF; ++t) {
    const int q = 16 * t + dq;
    AdvTraces nxt[4];
    if (t + 1 < TT::NTF) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (ew0 + 4 * v + de < mesh.K && q + 16 < TT::Nfc) gather(v, q + 16, nxt[v]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int le = 4 * v + de;
      const int64_t e = ew0 + le;
      double F = 0.0;
      if (e < mesh.K && q < TT::Nfc)
        F = adv_flux_from(cur[v], ops, ap, sX[wv * kEW + le], q / TT::Nfq, q);
      sQ[wv][le][dq] = F;
    }
    wave_sync_lds();
    const size_t pb = (size_t)t * 4 * NITP * 64 * KP;
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) {
      const double av = sQ[wv][row][4 * c2 + kq];
      dx2 pv;
#pragma unroll
      for (int u = 0; u < TT::NIT; ++u) {
        if (u % KP == 0) pv = load_pack(LfF + pb + ((size_t)c2 * NITP + u / KP) * 64 * KP);
        z[u] = M::mma(av, pv[u % KP], z[u]);
      }
    }
    wave_sync_lds();
#pragma unroll
    for (int v = 0; v < 4; ++v) cur[v] = nxt[v];
  }

  // inverse mass and LSRK stage
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int le = 4 * v + de;
    const int64_t e = ew0 + le;
    if (e >= mesh.K) continue;
    double jc[4];
    pyr_jac_coeffs(sX[wv * kEW + le], jc);
    const double dte = dt * mesh.mat[e * 4 + 3];
#pragma unroll
    for (int u = 0; u < TT::NIT; ++u) {
      const int i = 16 * u + dq;
      if (i >= TT::Np) continue;
      const double minv = 1.0 / (pyr_jac_eval(jc, ops.na[i], ops.nb[i]) * ops.wwc[i]);
      finish_coeff<MODE>(z[u][v], minv, 1.0, out, R, e * TT::Np + i, ra, rb, dte);
    }
  }
}

template <int N>
hipError_t adv_trace_n(const dgpyr_ctx& c, const double* U, double* T, hipStream_t s) {
  constexpr int G = N <= 4 ? 2 : 1;
  const int64_t nb = (c.K + kEB * G - 1) / (kEB * G);
  hipLaunchKernelGGL((k_adv_trace<N, G>), dim3((unsigned)nb), dim3(kBlock), 0, s, U, T, c.frag,
                     c.K);
  return hipGetLastError();
}

template <int N>
hipError_t adv_stage_n(const dgpyr_ctx& c, int mode, const double* U, const double* T,
                       double* out, double* R, double ra, double rb, double dt, hipStream_t s) {
  const int64_t nb = (c.K + kEB - 1) / kEB;
  if (mode == 0)
    hipLaunchKernelGGL((k_adv_stage<N, 0>), dim3((unsigned)nb), dim3(kBlock), 0, s, U, T, c.frag,
                       c.ops, c.mesh, c.adv, out, R, ra, rb, dt);
  else
    hipLaunchKernelGGL((k_adv_stage<N, 1>), dim3((unsigned)nb), dim3(kBlock), 0, s, U, T, c.frag,
                       c.ops, c.mesh, c.adv, out, R, ra, rb, dt);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_adv_trace(const dgpyr_ctx& c, const double* U, double* T, hipStream_t s) {
  switch (c.N) {
    case 0: return adv_trace_n<0>(c, U, T, s);
    case 1: return adv_trace_n<1>(c, U, T, s);
    case 2: return adv_trace_n<2>(c, U, T, s);
    case 3: return adv_trace_n<3>(c, U, T, s);
    case 4: return adv_trace_n<4>(c, U, T, s);
    case 5: return adv_trace_n<5>(c, U, T, s);
    case 6: return adv_trace_n<6>(c, U, T, s);
    case 7: return adv_trace_n<7>(c, U, T, s);
    case 8: return adv_trace_n<8>(c, U, T, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adv_stage(const dgpyr_ctx& c, int mode, const double* U, const double* T,
                            double* out, double* R, double ra, double rb, double dt,
                            hipStream_t s) {
  switch (c.N) {
    case 0: return adv_stage_n<0>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 1: return adv_stage_n<1>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 2: return adv_stage_n<2>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 3: return adv_stage_n<3>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 4: return adv_stage_n<4>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 5: return adv_stage_n<5>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 6: return adv_stage_n<6>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 7: return adv_stage_n<7>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 8: return adv_stage_n<8>(c, mode, U, T, out, R, ra, rb, dt, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dgpyr
