// Split-BF16 form of the fused stage: the volume derivative, volume projection
// and lift contractions run as three bf16 matrix-core products per multiply
// (hi*hi + hi*lo + lo*hi) with FP32 accumulation; traces, the pointwise
// metric, the flux, the inverse mass and the RK state stay in FP64.
// One wave owns 4 elements (rows i = 4 e + f); point tiles of 32 feed the
// 32-deep contractions.
#include <hip/hip_runtime.h>

#include "context.hpp"
#include "flux.hpp"
#include "geom.hpp"
#include "mfma.hpp"

namespace dgpyr {
namespace {

constexpr int kWaves = 4;
constexpr int kEW = 4;
constexpr int kEB = kWaves * kEW;
constexpr int kBlock = 64 * kWaves;

// Orders this wave's LDS writes before its later LDS reads (and reads before
// later writes): the transpose tile sQ[wv] is private to its wave and a
// wave's LDS operations complete in issue order, so no workgroup barrier is
// needed; the fences keep the compiler from moving LDS accesses across.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bfx8 load_bf8(const uint16_t* p) {
  return *reinterpret_cast<const bfx8*>(p);
}

// A operand pair from 8 FP64 values.
__device__ __forceinline__ void split8(const double* x, bfx8& hi, bfx8& lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    __bf16 h, l;
    split_bf16(x[j], h, l);
    hi[j] = h;
    lo[j] = l;
  }
}

// Neighbour of one element face: element, offset of its matching face in its
// trace row, row of the face-point permutation table, its rho c.
struct FaceNb {
  int nb, off, prow;
  double zp;
};

// Waves per SIMD the kernel is compiled for.  Unconstrained, N >= 6 takes
// more than 256 registers (with the accumulators) and runs one wave per
// SIMD; at two it fits without spilling up to N = 7 (17 registers spilled at
// N = 8) and runs 5.88 -> 3.56 ms (N = 6), 18.7 -> 12.1 ms (N = 7) and
// 31.7 -> 24.1 ms (N = 8) at 196608 pyramids.  Below N = 6 the unconstrained
// build already fits two or more.
template <int N>
struct Bf16Waves {
  static constexpr int value = N >= 6 ? 2 : 1;
};

// Unit face normals and surface Jacobians of the workgroup's elements in LDS
// ((N+1)^2 base points + 4 planar triangles per element), where they fit
// next to the transpose tiles under 56 KiB.
template <int N>
struct Bf16Norm {
  static constexpr int Nfq = (N + 1) * (N + 1);
  static constexpr int base = kEB * 16 * 8 + kWaves * 16 * 33 * 8 + kEB * 5 * 24 + 10 * Nfq * 4;
  static constexpr bool value = base + kEB * (Nfq + 4) * 4 * 8 <= 56 * 1024;
};

template <int N, int MODE>
__global__ __launch_bounds__(kBlock, Bf16Waves<N>::value) void k_stage_bf16(const double* U,
                                                       const double* __restrict__ T, Bf16Ops bo,
                                                       DevOps ops, DevMesh mesh, double* out,
                                                       double* R, double ra, double rb, double dt) {
  using TT = Tiles<N>;
  constexpr bool kNorm = Bf16Norm<N>::value;
  __shared__ double sX[kEB][16];
  __shared__ double sQ[kWaves][16][33];
  __shared__ FaceNb sNb[kEB][5];
  __shared__ int sPerm[10 * TT::Nfq];
  __shared__ double sN[kNorm ? kEB : 1][kNorm ? TT::Nfq + 4 : 1][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t eb0 = (int64_t)blockIdx.x * kEB;
  for (int x = threadIdx.x; x < kEB * 16; x += kBlock) {
    const int64_t e = eb0 + x / 16;
    sX[x / 16][x % 16] = e < mesh.K ? mesh.verts[e * 16 + (x % 16)] : 0.0;
  }
  for (int x = threadIdx.x; x < kEB * 5; x += kBlock) {
    const int le = x / 5, f = x - le * 5;
    const int64_t e = eb0 + le;
    FaceNb fn{-1, 0, 0, 0.0};
    if (e < mesh.K) {
      const int nb = mesh.conn[e * 8 + f];
      if (nb >= 0) {
        const int code = (mesh.conn[e * 8 + 5] >> (6 * f)) & 63;
        const int nf = code & 7, o = code >> 3;
        fn = FaceNb{nb, nf * TT::Nfq, (f == 0 ? o : 8 + o) * TT::Nfq,
                    mesh.mat[(int64_t)nb * 4 + 2]};
      }
    }
    sNb[le][f] = fn;
  }
  for (int x = threadIdx.x; x < 10 * TT::Nfq; x += kBlock) sPerm[x] = ops.perm[x];
  const int64_t ew0 = eb0 + wv * kEW;
  const int row = lane & 15, kq = lane >> 4;  // A: row, 8-wide k group
  const int de = lane >> 4, dq = lane & 15;   // D: element, column
  const int64_t e = ew0 + de;

  // A operands of U (rows 4 e + f): lane holds U[e][f][32c + 8 kq + j]
  bfx8 ah[TT::NCH32], al[TT::NCH32];
  {
    const int64_t ea = ew0 + (row >> 2);
    const int f = row & 3;
#pragma unroll
    for (int c = 0; c < TT::NCH32; ++c) {
      double x[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int n = 32 * c + 8 * kq + j;
        x[j] = (ea < mesh.K && n < TT::Np) ? U[(ea * 4 + f) * TT::Np + n] : 0.0;
      }
      split8(x, ah[c], al[c]);
    }
  }
  __syncthreads();
  if (kNorm) {
    // rows 0 .. Nfq-1: base points; Nfq + f - 1: triangle f = 1..4
    for (int x = threadIdx.x; x < kEB * (TT::Nfq + 4); x += kBlock) {
      const int le = x / (TT::Nfq + 4), r = x - le * (TT::Nfq + 4);
      const int f = r < TT::Nfq ? 0 : r - TT::Nfq + 1;
      const int q = r < TT::Nfq ? r : f * TT::Nfq;
      face_normal_unit(sX[le], f, ops.fa[q], ops.fb[q], sN[le][r]);
    }
    __syncthreads();
  }
  const double* xv = sX[wv * kEW + de];
  fx4 z[TT::NIT];
#pragma unroll
  for (int u = 0; u < TT::NIT; ++u) z[u] = fx4{0.f, 0.f, 0.f, 0.f};

  // volume (Algorithm 1): 32-point chunks of two 16-point derivative tiles
  for (int t32 = 0; t32 < TT::NT32C; ++t32) {
#pragma unroll
    for (int sub = 0; sub < 2; ++sub) {
      const int t = 2 * t32 + sub;
      fx4 yr = {0.f, 0.f, 0.f, 0.f}, ys = yr, yt = yr;
      if (t < TT::NTC) {
#pragma unroll
        for (int c = 0; c < TT::NCH32; ++c) {
          const size_t fo = (((size_t)t * TT::NCH32 + c) * 64 + lane) * 8;
          yr = mma_bf16x3(ah[c], al[c], load_bf8(bo.DrH + fo), load_bf8(bo.DrL + fo), yr);
          ys = mma_bf16x3(ah[c], al[c], load_bf8(bo.DsH + fo), load_bf8(bo.DsL + fo), ys);
          yt = mma_bf16x3(ah[c], al[c], load_bf8(bo.DtH + fo), load_bf8(bo.DtL + fo), yt);
        }
      }
      const int q = 16 * t + dq;
      double Q[4] = {0.0, 0.0, 0.0, 0.0};
      if (q < TT::Nc) {
        const int pm = q % TT::Nfq;
        double adj[9], J;
        pyr_metric(xv, ops.xg[pm % TT::n1], ops.xg[pm / TT::n1], adj, &J);
        const double w = ops.wv[q];
        double qp = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
          qp += adj[k] * (double)yr[1 + k] + adj[3 + k] * (double)ys[1 + k] +
                adj[6 + k] * (double)yt[1 + k];
        Q[0] = w * qp;
#pragma unroll
        for (int k = 0; k < 3; ++k)
          Q[1 + k] = w * (adj[k] * (double)yr[0] + adj[3 + k] * (double)ys[0] +
                          adj[6 + k] * (double)yt[0]);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) sQ[wv][4 * de + v][16 * sub + dq] = Q[v];
    }
    wave_lds_sync();
    bfx8 qh, ql;
    split8(&sQ[wv][row][8 * kq], qh, ql);
#pragma unroll
    for (int u = 0; u < TT::NIT; ++u) {
      const size_t fo = (((size_t)t32 * TT::NIT + u) * 64 + lane) * 8;
      z[u] = mma_bf16x3(qh, ql, load_bf8(bo.VH + fo), load_bf8(bo.VL + fo), z[u]);
    }
    wave_lds_sync();
  }

  // surface (Algorithm 2): fluxes of 32 face points per chunk; the traces of
  // chunk t + 1 are gathered while chunk t's fluxes and lift run.
  auto gather = [&](int q, FaceTraces& tr) {
    const int f = q / TT::Nfq, qq = q - f * TT::Nfq;
    const double* tm = T + (e * TT::Nfc + q) * 4;
    tr.pm = tm[0]; tr.um0 = tm[1]; tr.um1 = tm[2]; tr.um2 = tm[3];
    const FaceNb& fn = sNb[wv * kEW + de][f];
    tr.inner = fn.nb >= 0;
    if (tr.inner) {
      const double* tp = T + ((int64_t)fn.nb * TT::Nfc + fn.off + sPerm[fn.prow + qq]) * 4;
      tr.pp = tp[0]; tr.up0 = tp[1]; tr.up1 = tp[2]; tr.up2 = tp[3];
      tr.zp = fn.zp;
    }
  };
  const double zm = e < mesh.K ? mesh.mat[e * 4 + 2] : 0.0;
  FaceTraces cur[2];
#pragma unroll
  for (int sub = 0; sub < 2; ++sub)
    if (e < mesh.K && 16 * sub + dq < TT::Nfc) gather(16 * sub + dq, cur[sub]);
#pragma unroll
  for (int t32 = 0; t32 < TT::NT32F; ++t32) {
    FaceTraces nxt[2];
    if (t32 + 1 < TT::NT32F) {
#pragma unroll
      for (int sub = 0; sub < 2; ++sub) {
        const int q = 32 * (t32 + 1) + 16 * sub + dq;
        if (e < mesh.K && q < TT::Nfc) gather(q, nxt[sub]);
      }
    }
#pragma unroll
    for (int sub = 0; sub < 2; ++sub) {
      const int q = 32 * t32 + 16 * sub + dq;
      double F[4] = {0.0, 0.0, 0.0, 0.0};
      if (e < mesh.K && q < TT::Nfc) {
        const int f = q / TT::Nfq;
        if (kNorm) {
          const double* nr = sN[wv * kEW + de][f == 0 ? q : TT::Nfq + f - 1];
          flux_from_traces(cur[sub], mesh, zm, nr[0], nr[1], nr[2], ops.wf[q] * nr[3], F);
        } else {
          double nr[4];
          face_normal_unit(xv, f, ops.fa[q], ops.fb[q], nr);
          flux_from_traces(cur[sub], mesh, zm, nr[0], nr[1], nr[2], ops.wf[q] * nr[3], F);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) sQ[wv][4 * de + v][16 * sub + dq] = F[v];
    }
    wave_lds_sync();
    bfx8 fh, fl;
    split8(&sQ[wv][row][8 * kq], fh, fl);
#pragma unroll
    for (int u = 0; u < TT::NIT; ++u) {
      const size_t fo = (((size_t)t32 * TT::NIT + u) * 64 + lane) * 8;
      z[u] = mma_bf16x3(fh, fl, load_bf8(bo.LfH + fo), load_bf8(bo.LfL + fo), z[u]);
    }
    wave_lds_sync();
#pragma unroll
    for (int sub = 0; sub < 2; ++sub) cur[sub] = nxt[sub];
  }

  // inverse mass, material, RK stage (Algorithm 3)
  if (e >= mesh.K) return;
  const double kap = mesh.mat[e * 4 + 0], irho = mesh.mat[e * 4 + 1];
  const double dte = dt * mesh.mat[e * 4 + 3];
  double jc[4];  // J is bilinear in (a, b): four coefficients per element
  pyr_jac_coeffs(xv, jc);
#pragma unroll
  for (int u = 0; u < TT::NIT; ++u) {
    const int i = 16 * u + dq;
    if (i >= TT::Np) continue;
    const double minv = 1.0 / (pyr_jac_eval(jc, ops.na[i], ops.nb[i]) * ops.wwc[i]);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double acc = (double)z[u][v] - (v == 0 ? source_term<TT::Np>(mesh, e, i) : 0.0);
      finish_coeff<MODE>(acc, minv, v == 0 ? kap : irho, out, R, (e * 4 + v) * TT::Np + i, ra,
                         rb, dte);
    }
  }
}

template <int N>
hipError_t stage_bf16_n(const dgpyr_ctx& c, int mode, const double* U, const double* T,
                        double* out, double* R, double ra, double rb, double dt, hipStream_t s) {
  const int64_t nb = (c.K + kEB - 1) / kEB;
  if (mode == 0)
    hipLaunchKernelGGL((k_stage_bf16<N, 0>), dim3((unsigned)nb), dim3(kBlock), 0, s, U, T, c.bf,
                       c.ops, c.mesh, out, R, ra, rb, dt);
  else
    hipLaunchKernelGGL((k_stage_bf16<N, 1>), dim3((unsigned)nb), dim3(kBlock), 0, s, U, T, c.bf,
                       c.ops, c.mesh, out, R, ra, rb, dt);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stage_bf16(const dgpyr_ctx& c, int mode, const double* U, const double* T,
                             double* out, double* R, double ra, double rb, double dt,
                             hipStream_t s) {
  switch (c.N) {
    case 0: return stage_bf16_n<0>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 1: return stage_bf16_n<1>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 2: return stage_bf16_n<2>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 3: return stage_bf16_n<3>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 4: return stage_bf16_n<4>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 5: return stage_bf16_n<5>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 6: return stage_bf16_n<6>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 7: return stage_bf16_n<7>(c, mode, U, T, out, R, ra, rb, dt, s);
    case 8: return stage_bf16_n<8>(c, mode, U, T, out, R, ra, rb, dt, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dgpyr
