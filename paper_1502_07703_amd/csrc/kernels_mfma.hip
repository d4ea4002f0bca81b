// Matrix-core kernels: the volume term (Algorithm 1) as two chained
// contractions per wave with the pointwise metric between them, the trace
// interpolation, and the surface lift + inverse mass + LSRK update
// (Algorithms 2-3).  One wave owns 4 elements; a workgroup of 4 waves owns 16.
#include <hip/hip_runtime.h>

#include "context.hpp"
#include "flux.hpp"
#include "geom.hpp"
#include "mfma.hpp"

namespace dgpyr {
namespace {

constexpr int kWaves = 4;
constexpr int kEW = 4;                 // elements per wave
constexpr int kEB = kWaves * kEW;      // elements per workgroup
constexpr int kBlock = 64 * kWaves;

// Orders this wave's LDS writes before its later LDS reads (and reads before
// later writes).  A wave's LDS operations complete in issue order, so data
// exchanged between lanes of one wave needs no workgroup barrier; the fences
// keep the compiler from moving LDS accesses across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A operands of U for this wave: lane l holds U[e][f][4c + l/16] with (e, f)
// the element and field of row l % 16 in the form's row order; zero beyond Np
// or beyond the mesh.
template <int N, int FORM>
__device__ __forceinline__ void load_u_frags(const double* U, int64_t ew0, int64_t K,
                                             int lane, typename Mma<FORM>::T* afr) {
  using TT = Tiles<N>;
  const int row = lane & 15, kq = lane >> 4;
  const int64_t e = ew0 + Mma<FORM>::row_elem(row);
  const int f = Mma<FORM>::row_field(row);
  const double* src = U + (e * 4 + f) * TT::Np;
#pragma unroll
  for (int c = 0; c < TT::NCH; ++c) {
    const int n = 4 * c + kq;
    afr[c] = (e < K && n < TT::Np) ? (typename Mma<FORM>::T)src[n] : (typename Mma<FORM>::T)0;
  }
}

// Volume term: Y_rho = D_rho U at 16 cubature points per tile (3 contractions),
// then Q_p = w sum_rho,k adj[rho][k] d_rho u_k, Q_u_k = w sum_rho adj[rho][k] d_rho p
// in FP64, then vol += V^T Q.  adj = J d(r,s,t)/dx is evaluated from the
// element's vertices at the point's (a, b) (it is constant along c).
template <int N, int FORM>
__global__ __launch_bounds__(kBlock) void k_volume_mfma(const double* __restrict__ U,
                                                        double* __restrict__ vol, FragOps fo,
                                                        DevOps ops, DevMesh mesh) {
  using TT = Tiles<N>;
  using M = Mma<FORM>;
  using T = typename M::T;
  __shared__ double sX[kEB][16];
  __shared__ T sQ[kWaves][16][17];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t eb0 = (int64_t)blockIdx.x * kEB;
  for (int x = threadIdx.x; x < kEB * 16; x += kBlock) {
    const int64_t e = eb0 + x / 16;
    sX[x / 16][x % 16] = e < mesh.K ? mesh.verts[e * 16 + (x % 16)] : 0.0;
  }
  const int64_t ew0 = eb0 + wv * kEW;
  T afr[TT::NCH];
  load_u_frags<N, FORM>(U, ew0, mesh.K, lane, afr);
  __syncthreads();

  constexpr int KP = Pack<T>::KP;
  constexpr int NCHP = (TT::NCH + KP - 1) / KP, NITP = (TT::NIT + KP - 1) / KP;
  using PV = typename Pack<T>::V;
  const T* DrF = static_cast<const T*>(fo.DrF) + lane * KP;
  const T* DsF = static_cast<const T*>(fo.DsF) + lane * KP;
  const T* DtF = static_cast<const T*>(fo.DtF) + lane * KP;
  const T* VF = static_cast<const T*>(fo.VF) + lane * KP;
  const int de = lane >> 4, dq = lane & 15;
  const int row = lane & 15, kq = lane >> 4;
  const double* xv = sX[wv * kEW + de];
  typename M::Acc z[TT::NIT];
#pragma unroll
  for (int u = 0; u < TT::NIT; ++u) z[u] = M::zero();

  for (int t = 0; t < TT::NTC; ++t) {
    typename M::Acc yr = M::zero(), ys = M::zero(), yt = M::zero();
    const size_t fb = (size_t)t * NCHP * 64 * KP;
    PV pr, ps, pt;
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
      // keep at most four chunks of operand loads in flight: hoisting all of
      // them costs enough registers to halve the occupancy
      if ((c & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    const int q = 16 * t + dq;
    double Q0 = 0.0, Q1 = 0.0, Q2 = 0.0, Q3 = 0.0;
    if (q < TT::Nc) {
      const int pm = q % TT::Nfq;
      double adj[9], J;
      pyr_metric(xv, ops.xg[pm % TT::n1], ops.xg[pm / TT::n1], adj, &J);
      const double w = ops.wv[q];
      const double d[3][4] = {{(double)yr[0], (double)yr[1], (double)yr[2], (double)yr[3]},
                              {(double)ys[0], (double)ys[1], (double)ys[2], (double)ys[3]},
                              {(double)yt[0], (double)yt[1], (double)yt[2], (double)yt[3]}};
      double qp = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) qp += adj[3 * r + k] * d[r][1 + k];
      Q0 = w * qp;
      Q1 = w * (adj[0] * d[0][0] + adj[3] * d[1][0] + adj[6] * d[2][0]);
      Q2 = w * (adj[1] * d[0][0] + adj[4] * d[1][0] + adj[7] * d[2][0]);
      Q3 = w * (adj[2] * d[0][0] + adj[5] * d[1][0] + adj[8] * d[2][0]);
    }
    // D layout (element de, point dq, 4 fields) -> A layout (row (e, f), point k)
    sQ[wv][M::row(de, 0)][dq] = (T)Q0;
    sQ[wv][M::row(de, 1)][dq] = (T)Q1;
    sQ[wv][M::row(de, 2)][dq] = (T)Q2;
    sQ[wv][M::row(de, 3)][dq] = (T)Q3;
    __syncthreads();
    const size_t pb = (size_t)t * 4 * NITP * 64 * KP;
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) {
      const T a = sQ[wv][row][4 * c2 + kq];
      PV pv;
#pragma unroll
      for (int u = 0; u < TT::NIT; ++u) {
        if (u % KP == 0) pv = load_pack(VF + pb + ((size_t)c2 * NITP + u / KP) * 64 * KP);
        z[u] = M::mma(a, pv[u % KP], z[u]);
      }
    }
    __syncthreads();
  }
  const int64_t e = ew0 + de;
  if (e < mesh.K) {
    double* o = vol + e * 4 * TT::Np;
#pragma unroll
    for (int u = 0; u < TT::NIT; ++u) {
      const int i = 16 * u + dq;
      if (i < TT::Np) {
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v * TT::Np + i] = (double)z[u][v];
      }
    }
  }
}

// Trace interpolation U^f = V^f U at every face point (FP64 in every form:
// jumps of traces are differences of O(1) values).  A wave owns G groups of 4
// elements; each operator fragment loaded feeds G matrix-core products.  Lane
// l ends with all four fields of element 4g + l/16 at face point 16t + l%16
// and stores them as one 32-byte vector into T[K][Nfc][4].
template <int N, int G>
__global__ __launch_bounds__(kBlock) void k_trace_mfma(const double* __restrict__ U,
                                                       double* __restrict__ T, FragOps fo,
                                                       int64_t K) {
  using TT = Tiles<N>;
  using M = Mma<0>;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t ew0 = (int64_t)blockIdx.x * (kEB * G) + wv * (kEW * G);
  double afr[G][TT::NCH];
#pragma unroll
  for (int g = 0; g < G; ++g) load_u_frags<N, 0>(U, ew0 + kEW * g, K, lane, afr[g]);
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
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t e = ew0 + kEW * g + de;
      if (e < K && q < TT::Nfc) *reinterpret_cast<dx4*>(T + (e * TT::Nfc + q) * 4) = y[g];
    }
  }
}

// Surface term, inverse mass and LSRK update.  Per 16-point face tile each
// lane evaluates the FP64 flux of one (element, face point); the fluxes are
// transposed through LDS into A operands and lifted by L = V^f^T F on the
// matrix cores; the epilogue adds the volume term and applies M^-1, the
// material factors and the RK stage.
template <int N, int FORM, int MODE>
__global__ __launch_bounds__(kBlock) void k_surface_mfma(const double* __restrict__ T,
                                                         const double* __restrict__ vol,
                                                         FragOps fo, DevOps ops, DevMesh mesh,
                                                         double* out, double* R, double ra,
                                                         double rb, double dt) {
  using TT = Tiles<N>;
  using M = Mma<FORM>;
  using TV = typename M::T;
  __shared__ double sX[kEB][16];
  __shared__ TV sF[kWaves][16][17];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t eb0 = (int64_t)blockIdx.x * kEB;
  for (int x = threadIdx.x; x < kEB * 16; x += kBlock) {
    const int64_t e = eb0 + x / 16;
    sX[x / 16][x % 16] = e < mesh.K ? mesh.verts[e * 16 + (x % 16)] : 0.0;
  }
  __syncthreads();
  const int64_t ew0 = eb0 + wv * kEW;
  const int de = lane >> 4, dq = lane & 15;
  const int row = lane & 15, kq = lane >> 4;
  const int64_t e = ew0 + de;
  const double* xv = sX[wv * kEW + de];
  constexpr int KP = Pack<TV>::KP;
  constexpr int NITP = (TT::NIT + KP - 1) / KP;
  using PV = typename Pack<TV>::V;
  const TV* LfF = static_cast<const TV*>(fo.LfF) + lane * KP;
  typename M::Acc z[TT::NIT];
#pragma unroll
  for (int u = 0; u < TT::NIT; ++u) z[u] = M::zero();
  for (int t = 0; t < TT::NTF; ++t) {
    const int q = 16 * t + dq;
    double F[4] = {0.0, 0.0, 0.0, 0.0};
    if (e < mesh.K && q < TT::Nfc) face_flux<TT::Nfq>(T, ops, mesh, xv, e, q, F);
#pragma unroll
    for (int v = 0; v < 4; ++v) sF[wv][M::row(de, v)][dq] = (TV)F[v];
    __syncthreads();
    const size_t pb = (size_t)t * 4 * NITP * 64 * KP;
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) {
      const TV a = sF[wv][row][4 * c2 + kq];
      PV pv;
#pragma unroll
      for (int u = 0; u < TT::NIT; ++u) {
        if (u % KP == 0) pv = load_pack(LfF + pb + ((size_t)c2 * NITP + u / KP) * 64 * KP);
        z[u] = M::mma(a, pv[u % KP], z[u]);
      }
    }
    __syncthreads();
  }
  if (e >= mesh.K) return;
  const double kap = mesh.mat[e * 4 + 0], irho = mesh.mat[e * 4 + 1];
  const double dte = dt * mesh.mat[e * 4 + 3];
  const double* vo = vol + e * 4 * TT::Np;
#pragma unroll
  for (int u = 0; u < TT::NIT; ++u) {
    const int i = 16 * u + dq;
    if (i >= TT::Np) continue;
    const double minv = 1.0 / (pyr_jac(xv, ops.na[i], ops.nb[i]) * ops.wwc[i]);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t idx = (e * 4 + v) * TT::Np + i;
      const double acc = vo[v * TT::Np + i] + (double)z[u][v] -
                         (v == 0 ? source_term<TT::Np>(mesh, e, i) : 0.0);
      finish_coeff<MODE>(acc, minv, v == 0 ? kap : irho, out, R, idx, ra, rb, dte);
    }
  }
}

// Fused stage: volume term and surface lift accumulate into the same
// matrix-core accumulators, then inverse mass, material and the RK stage are
// applied in the epilogue; the volume contribution never leaves registers.
// A wave owns G groups of 4 elements: every operator fragment loaded feeds G
// products.  The D -> A layout changes go through a per-wave LDS tile and need
// only wave-local ordering.  In RK mode the kernel reads and writes only its
// own elements' U and R; other workgroups read traces (T), never U, so the
// in-place update is safe.  In RK mode out is U itself, so U is not declared
// __restrict__ in the stage kernels.
// Waves per SIMD the fused stage kernel is compiled for (register budget
// 512 / waves).  Mostly the largest count that holds the kernel without
// spilling (gfx950 build: FP64 N = 4, one group: 150 registers for three
// waves against 200 when unconstrained; FP64 N = 6: 236 for two waves against
// 312).  FP64 N = 7 and 8 with one group spill at two waves (58 and 284
// registers) and are still faster there than at one wave: 63.0 -> 48.4 ms
// (N = 7, 384000 pyramids) and 66.6 -> 61.0 ms (N = 8, 196608 pyramids),
// whereas N = 5 at three waves (38 spilled) is slower, 3.66 -> 3.92 ms.
template <int N, int FORM, int G>
struct StageWaves {
  static constexpr int value =
      G == 2 ? (FORM == 0 ? (N <= 4 ? 2 : 1) : (N <= 6 ? 2 : 1))
             : (FORM == 0 ? (N <= 4 ? 3 : 2) : (N <= 6 ? 3 : 2));
};

// The face normals of an element are few: the base face's vary with (a, b),
// the four triangles are planar, so there are (N+1)^2 + 4 distinct unit
// normals (with their surface Jacobians).  The stage kernel evaluates them
// once per element into LDS, which saves a normal, a square root and three
// divisions per flux evaluation, where the table keeps the workgroup within
// 52 KiB of LDS (three workgroups per CU).  With the tables of the faces'
// neighbours (element, matching face, permutation row, rho c) and of the
// face-point permutations beside it, the surface loop gathers the traces of
// tile t + 1 while tile t's flux and lift run: measured at 384000 pyramids,
// N = 4, stage 3.09 -> 2.92 ms (N = 6, 196608 pyramids: 7.68 -> 7.38 ms) in
// a same-device comparison.
template <int N, int FORM, int G>
struct NormalTable {
  static constexpr int EB = kWaves * kEW * G;
  static constexpr int Nfq = (N + 1) * (N + 1);
  static constexpr int base =
      EB * 16 * 8 + kWaves * G * 16 * 17 * (FORM == 0 ? 8 : 4);  // sX, sQ
  static constexpr int bytes = EB * (Nfq + 4) * 4 * 8 + EB * 5 * 24 + 10 * Nfq * 4;
  static constexpr bool value = base + bytes <= 52 * 1024;
};

// Neighbour of one element face for the trace gathers: element, offset of
// its matching face in its trace row, row of the face-point permutation
// table, and its rho c.
struct FaceNb {
  int nb, off, prow;
  double zp;
};

template <int N, int FORM, int MODE, int G>
__global__ __launch_bounds__(kBlock, (StageWaves<N, FORM, G>::value)) void k_stage_mfma(const double* U,
                                                       const double* __restrict__ T, FragOps fo,
                                                       DevOps ops, DevMesh mesh, double* out,
                                                       double* R, double ra, double rb, double dt) {
  using TT = Tiles<N>;
  using M = Mma<FORM>;
  using TV = typename M::T;
  constexpr int EW = kEW * G;      // elements per wave
  constexpr int EB = kWaves * EW;  // elements per workgroup
  constexpr bool kNorm = NormalTable<N, FORM, G>::value;
  __shared__ double sX[EB][16];
  __shared__ TV sQ[kWaves][G][16][17];
  __shared__ double sN[kNorm ? EB : 1][kNorm ? TT::Nfq + 4 : 1][4];
  __shared__ FaceNb sNb[kNorm ? EB : 1][5];
  __shared__ int sPerm[kNorm ? 10 * TT::Nfq : 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t eb0 = (int64_t)blockIdx.x * EB;
  for (int x = threadIdx.x; x < EB * 16; x += kBlock) {
    const int64_t e = eb0 + x / 16;
    sX[x / 16][x % 16] = e < mesh.K ? mesh.verts[e * 16 + (x % 16)] : 0.0;
  }
  const int64_t ew0 = eb0 + wv * EW;
  TV afr[G][TT::NCH];
#pragma unroll
  for (int g = 0; g < G; ++g) load_u_frags<N, FORM>(U, ew0 + kEW * g, mesh.K, lane, afr[g]);
  __syncthreads();
  if (kNorm) {
    // rows 0 .. Nfq-1: base-face points; Nfq + f - 1: triangle f = 1..4
    for (int x = threadIdx.x; x < EB * (TT::Nfq + 4); x += kBlock) {
      const int le = x / (TT::Nfq + 4), r = x - le * (TT::Nfq + 4);
      const int f = r < TT::Nfq ? 0 : r - TT::Nfq + 1;
      const int q = r < TT::Nfq ? r : f * TT::Nfq;
      face_normal_unit(sX[le], f, ops.fa[q], ops.fb[q], sN[le][r]);
    }
    for (int x = threadIdx.x; x < EB * 5; x += kBlock) {
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
    __syncthreads();
  }

  constexpr int KP = Pack<TV>::KP;
  constexpr int NCHP = (TT::NCH + KP - 1) / KP, NITP = (TT::NIT + KP - 1) / KP;
  using PV = typename Pack<TV>::V;
  const TV* DrF = static_cast<const TV*>(fo.DrF) + lane * KP;
  const TV* DsF = static_cast<const TV*>(fo.DsF) + lane * KP;
  const TV* DtF = static_cast<const TV*>(fo.DtF) + lane * KP;
  const TV* VF = static_cast<const TV*>(fo.VF) + lane * KP;
  const TV* LfF = static_cast<const TV*>(fo.LfF) + lane * KP;
  const int de = lane >> 4, dq = lane & 15;
  const int row = lane & 15, kq = lane >> 4;
  typename M::Acc z[G][TT::NIT];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int u = 0; u < TT::NIT; ++u) z[g][u] = M::zero();

  // volume (Algorithm 1)
  for (int t = 0; t < TT::NTC; ++t) {
    typename M::Acc yr[G], ys[G], yt[G];
#pragma unroll
    for (int g = 0; g < G; ++g) yr[g] = ys[g] = yt[g] = M::zero();
    const size_t fb = (size_t)t * NCHP * 64 * KP;
    PV pr, ps, pt;
#pragma unroll
    for (int c = 0; c < TT::NCH; ++c) {
      if (c % KP == 0) {
        const size_t o = fb + (size_t)(c / KP) * 64 * KP;
        pr = load_pack(DrF + o);
        ps = load_pack(DsF + o);
        pt = load_pack(DtF + o);
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        yr[g] = M::mma(afr[g][c], pr[c % KP], yr[g]);
        ys[g] = M::mma(afr[g][c], ps[c % KP], ys[g]);
        yt[g] = M::mma(afr[g][c], pt[c % KP], yt[g]);
      }
      // keep at most a few chunks of operand loads in flight: hoisting all of
      // them costs enough registers to halve the occupancy
      if ((c & (4 / G - 1)) == 4 / G - 1) __builtin_amdgcn_sched_barrier(0);
    }
    const int q = 16 * t + dq;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      double Q[4] = {0.0, 0.0, 0.0, 0.0};
      if (q < TT::Nc) {
        const double* xv = sX[wv * EW + kEW * g + de];
        const int pm = q % TT::Nfq;
        double adj[9], J;
        pyr_metric(xv, ops.xg[pm % TT::n1], ops.xg[pm / TT::n1], adj, &J);
        const double w = ops.wv[q];
        double dr[4], ds[4], dtt[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          dr[v] = (double)yr[g][v];
          ds[v] = (double)ys[g][v];
          dtt[v] = (double)yt[g][v];
        }
        double qp = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k)
          qp += adj[k] * dr[1 + k] + adj[3 + k] * ds[1 + k] + adj[6 + k] * dtt[1 + k];
        Q[0] = w * qp;
#pragma unroll
        for (int k = 0; k < 3; ++k)
          Q[1 + k] = w * (adj[k] * dr[0] + adj[3 + k] * ds[0] + adj[6 + k] * dtt[0]);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) sQ[wv][g][M::row(de, v)][dq] = (TV)Q[v];
    }
    wave_lds_sync();
    const size_t pb = (size_t)t * 4 * NITP * 64 * KP;
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) {
      TV a[G];
#pragma unroll
      for (int g = 0; g < G; ++g) a[g] = sQ[wv][g][row][4 * c2 + kq];
      PV pv;
#pragma unroll
      for (int u = 0; u < TT::NIT; ++u) {
        if (u % KP == 0) pv = load_pack(VF + pb + ((size_t)c2 * NITP + u / KP) * 64 * KP);
#pragma unroll
        for (int g = 0; g < G; ++g) z[g][u] = M::mma(a[g], pv[u % KP], z[g][u]);
      }
    }
    wave_lds_sync();
  }

  // surface (Algorithm 2).  With the LDS tables the traces of tile t + 1 are
  // gathered while tile t's flux and lift run.
  auto gather = [&](int g, int q, FaceTraces& tr) {
    const int64_t e = ew0 + kEW * g + de;
    const int f = q / TT::Nfq, qq = q - f * TT::Nfq;
    const double* tm = T + (e * TT::Nfc + q) * 4;
    tr.pm = tm[0]; tr.um0 = tm[1]; tr.um1 = tm[2]; tr.um2 = tm[3];
    const FaceNb& fn = sNb[wv * EW + kEW * g + de][f];
    tr.inner = fn.nb >= 0;
    if (tr.inner) {
      const double* tp = T + ((int64_t)fn.nb * TT::Nfc + fn.off + sPerm[fn.prow + qq]) * 4;
      tr.pp = tp[0]; tr.up0 = tp[1]; tr.up1 = tp[2]; tr.up2 = tp[3];
      tr.zp = fn.zp;
    }
  };
  FaceTraces cur[G];
  if (kNorm) {
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (ew0 + kEW * g + de < mesh.K && dq < TT::Nfc) gather(g, dq, cur[g]);
  }
#pragma unroll
  for (int t = 0; t < TT::NTF; ++t) {
    const int q = 16 * t + dq;
    FaceTraces nxt[G];
    if (kNorm && t + 1 < TT::NTF) {
#pragma unroll
      for (int g = 0; g < G; ++g)
        if (ew0 + kEW * g + de < mesh.K && q + 16 < TT::Nfc) gather(g, q + 16, nxt[g]);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t e = ew0 + kEW * g + de;
      double F[4] = {0.0, 0.0, 0.0, 0.0};
      if (e < mesh.K && q < TT::Nfc) {
        if (kNorm) {
          const int f = q / TT::Nfq;
          const double* nr = sN[wv * EW + kEW * g + de][f == 0 ? q : TT::Nfq + f - 1];
          flux_from_traces(cur[g], mesh, mesh.mat[e * 4 + 2], nr[0], nr[1], nr[2],
                           ops.wf[q] * nr[3], F);
        } else {
          face_flux<TT::Nfq>(T, ops, mesh, sX[wv * EW + kEW * g + de], e, q, F);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) sQ[wv][g][M::row(de, v)][dq] = (TV)F[v];
    }
    wave_lds_sync();
    const size_t pb = (size_t)t * 4 * NITP * 64 * KP;
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) {
      TV a[G];
#pragma unroll
      for (int g = 0; g < G; ++g) a[g] = sQ[wv][g][row][4 * c2 + kq];
      PV pv;
#pragma unroll
      for (int u = 0; u < TT::NIT; ++u) {
        if (u % KP == 0) pv = load_pack(LfF + pb + ((size_t)c2 * NITP + u / KP) * 64 * KP);
#pragma unroll
        for (int g = 0; g < G; ++g) z[g][u] = M::mma(a[g], pv[u % KP], z[g][u]);
      }
    }
    wave_lds_sync();
    if (kNorm) {
#pragma unroll
      for (int g = 0; g < G; ++g) cur[g] = nxt[g];
    }
  }

  // inverse mass, material, RK stage (Algorithm 3)
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int64_t e = ew0 + kEW * g + de;
    if (e >= mesh.K) continue;
    double jc[4];
    pyr_jac_coeffs(sX[wv * EW + kEW * g + de], jc);
    const double kap = mesh.mat[e * 4 + 0], irho = mesh.mat[e * 4 + 1];
    const double dte = dt * mesh.mat[e * 4 + 3];
#pragma unroll
    for (int u = 0; u < TT::NIT; ++u) {
      const int i = 16 * u + dq;
      if (i >= TT::Np) continue;
      const double minv = 1.0 / (pyr_jac_eval(jc, ops.na[i], ops.nb[i]) * ops.wwc[i]);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double acc = (double)z[g][u][v] - (v == 0 ? source_term<TT::Np>(mesh, e, i) : 0.0);
        finish_coeff<MODE>(acc, minv, v == 0 ? kap : irho, out, R, (e * 4 + v) * TT::Np + i,
                           ra, rb, dte);
      }
    }
  }
}

// Fused stage with the operator fragments of each tile staged in LDS once per
// workgroup: the four waves share every fragment instead of each streaming it
// from L2 (the vector-memory address unit was the stage kernel's limiter).
// Per volume tile the workgroup copies the derivative and projection
// fragments of that tile (16 bytes per thread and load) between two
// barriers, then every wave reads its B operands from LDS; the surface tiles
// stage the lift fragments the same way.  One 4-element group per wave.
template <int N, int FORM>
struct StagedDims {
  using TT = Tiles<N>;
  using TV = typename Mma<FORM>::T;
  static constexpr int KP = Pack<TV>::KP;
  static constexpr int NCHP = (TT::NCH + KP - 1) / KP;
  static constexpr int NITP = (TT::NIT + KP - 1) / KP;
  static constexpr int DPACKS = NCHP * 64;   // packs of one derivative operator per tile
  static constexpr int PPACKS = 4 * NITP * 64;  // packs of a projection / lift tile
  static constexpr int PACKS = 3 * DPACKS + PPACKS;
  static constexpr int BYTES = PACKS * 16;
  // fits one workgroup's LDS next to the vertex, transpose, face-neighbour and
  // face-point permutation tiles, under 64 KiB
  static constexpr bool fits = BYTES + kEB * 16 * 8 + kWaves * 16 * 17 * 8 + kEB * 5 * 24 +
                                   10 * TT::Nfq * 4 <= 65536;
};

template <int N, int FORM, int MODE>
__global__ __launch_bounds__(kBlock, (StageWaves<N, FORM, 1>::value)) void k_stage_staged(
    const double* U, const double* __restrict__ T, FragOps fo, DevOps ops,
    DevMesh mesh, double* out, double* R, double ra, double rb, double dt) {
  using TT = Tiles<N>;
  using M = Mma<FORM>;
  using TV = typename M::T;
  using SD = StagedDims<N, FORM>;
  constexpr int KP = SD::KP, NCHP = SD::NCHP, NITP = SD::NITP;
  using PV = typename Pack<TV>::V;
  __shared__ double sX[kEB][16];
  __shared__ TV sQ[kWaves][16][17];
  __shared__ PV sB[SD::PACKS];  // [Dr | Ds | Dt][NCHP][64], then [4][NITP][64]
  __shared__ FaceNb sNb[kEB][5];
  __shared__ int sPerm[10 * TT::Nfq];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t eb0 = (int64_t)blockIdx.x * kEB;
  for (int x = threadIdx.x; x < kEB * 16; x += kBlock) {
    const int64_t e = eb0 + x / 16;
    sX[x / 16][x % 16] = e < mesh.K ? mesh.verts[e * 16 + (x % 16)] : 0.0;
  }
  // face neighbours and face-point permutations (visible after the first
  // barrier of the volume loop)
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
  TV afr[TT::NCH];
  load_u_frags<N, FORM>(U, ew0, mesh.K, lane, afr);

  const PV* DrF = reinterpret_cast<const PV*>(fo.DrF);
  const PV* DsF = reinterpret_cast<const PV*>(fo.DsF);
  const PV* DtF = reinterpret_cast<const PV*>(fo.DtF);
  const PV* VF = reinterpret_cast<const PV*>(fo.VF);
  const PV* LfF = reinterpret_cast<const PV*>(fo.LfF);
  const int de = lane >> 4, dq = lane & 15;
  const int row = lane & 15, kq = lane >> 4;
  const int64_t e = ew0 + de;
  const double* xv = sX[wv * kEW + de];
  typename M::Acc z[TT::NIT];
#pragma unroll
  for (int u = 0; u < TT::NIT; ++u) z[u] = M::zero();

  // volume (Algorithm 1)
  for (int t = 0; t < TT::NTC; ++t) {
    __syncthreads();  // previous tile's readers are done with sB
    for (int x = threadIdx.x; x < SD::PACKS; x += kBlock) {
      const int op = x / SD::DPACKS;
      const int r = x - op * SD::DPACKS;
      sB[x] = op == 0   ? DrF[(size_t)t * SD::DPACKS + r]
              : op == 1 ? DsF[(size_t)t * SD::DPACKS + r]
              : op == 2 ? DtF[(size_t)t * SD::DPACKS + r]
                        : VF[(size_t)t * SD::PPACKS + (x - 3 * SD::DPACKS)];
    }
    __syncthreads();
    typename M::Acc yr = M::zero(), ys = M::zero(), yt = M::zero();
    PV pr, ps, pt;
#pragma unroll
    for (int c = 0; c < TT::NCH; ++c) {
      if (c % KP == 0) {
        const int o = (c / KP) * 64 + lane;
        pr = sB[o];
        ps = sB[SD::DPACKS + o];
        pt = sB[2 * SD::DPACKS + o];
      }
      yr = M::mma(afr[c], pr[c % KP], yr);
      ys = M::mma(afr[c], ps[c % KP], ys);
      yt = M::mma(afr[c], pt[c % KP], yt);
    }
    const int q = 16 * t + dq;
    double Q[4] = {0.0, 0.0, 0.0, 0.0};
    if (q < TT::Nc) {
      const int pm = q % TT::Nfq;
      double adj[9], J;
      pyr_metric(xv, ops.xg[pm % TT::n1], ops.xg[pm / TT::n1], adj, &J);
      const double w = ops.wv[q];
      double dr[4], ds[4], dtt[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        dr[v] = (double)yr[v];
        ds[v] = (double)ys[v];
        dtt[v] = (double)yt[v];
      }
      double qp = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        qp += adj[k] * dr[1 + k] + adj[3 + k] * ds[1 + k] + adj[6 + k] * dtt[1 + k];
      Q[0] = w * qp;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        Q[1 + k] = w * (adj[k] * dr[0] + adj[3 + k] * ds[0] + adj[6 + k] * dtt[0]);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) sQ[wv][M::row(de, v)][dq] = (TV)Q[v];
    wave_lds_sync();
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) {
      const TV a = sQ[wv][row][4 * c2 + kq];
      PV pv;
#pragma unroll
      for (int u = 0; u < TT::NIT; ++u) {
        if (u % KP == 0) pv = sB[3 * SD::DPACKS + (c2 * NITP + u / KP) * 64 + lane];
        z[u] = M::mma(a, pv[u % KP], z[u]);
      }
    }
    wave_lds_sync();
  }

  // surface (Algorithm 2): the traces of tile t + 1 are gathered while tile
  // t's flux, lift staging and lift run.
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
  FaceTraces cur;
  if (e < mesh.K && dq < TT::Nfc) gather(dq, cur);
#pragma unroll
  for (int t = 0; t < TT::NTF; ++t) {
    const int q = 16 * t + dq;
    FaceTraces nxt;
    if (t + 1 < TT::NTF && e < mesh.K && q + 16 < TT::Nfc) gather(q + 16, nxt);
    double F[4] = {0.0, 0.0, 0.0, 0.0};
    if (e < mesh.K && q < TT::Nfc) {
      double nr[4];
      face_normal_unit(xv, q / TT::Nfq, ops.fa[q], ops.fb[q], nr);
      flux_from_traces(cur, mesh, mesh.mat[e * 4 + 2], nr[0], nr[1], nr[2], ops.wf[q] * nr[3], F);
    }
    __syncthreads();
    for (int x = threadIdx.x; x < SD::PPACKS; x += kBlock) sB[x] = LfF[(size_t)t * SD::PPACKS + x];
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) sQ[wv][M::row(de, v)][dq] = (TV)F[v];
    wave_lds_sync();
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) {
      const TV a = sQ[wv][row][4 * c2 + kq];
      PV pv;
#pragma unroll
      for (int u = 0; u < TT::NIT; ++u) {
        if (u % KP == 0) pv = sB[(c2 * NITP + u / KP) * 64 + lane];
        z[u] = M::mma(a, pv[u % KP], z[u]);
      }
    }
    wave_lds_sync();
    cur = nxt;
  }

  // inverse mass, material, RK stage (Algorithm 3)
  if (e >= mesh.K) return;
  double jc[4];
  pyr_jac_coeffs(xv, jc);
  const double kap = mesh.mat[e * 4 + 0], irho = mesh.mat[e * 4 + 1];
  const double dte = dt * mesh.mat[e * 4 + 3];
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

// Element groups per wave of the fused stage (1 or 2, set per context) and of
// the trace (default by N; measured at 384000 pyramids, N = 4: 0.82 ms with
// one group, 0.74 ms with two, 0.62 ms with four; four groups at N = 5 and
// two at N >= 6 need more registers than leave several waves per SIMD).
inline int mfma_groups(const dgpyr_ctx& c) { return c.mfma_groups == 2 ? 2 : 1; }
inline int trace_groups(const dgpyr_ctx& c) {
  if (c.trace_groups == 1 || c.trace_groups == 2 || c.trace_groups == 4) return c.trace_groups;
  return c.N <= 4 ? 4 : c.N == 5 ? 2 : 1;
}

template <int N, int FORM, int G>
hipError_t stage_mfma_n(const dgpyr_ctx& c, int mode, const double* U, const double* T, double* out,
                        double* R, double ra, double rb, double dt, hipStream_t s) {
  const int64_t nb = (c.K + kEB * G - 1) / (kEB * G);
  if (mode == 0)
    hipLaunchKernelGGL((k_stage_mfma<N, FORM, 0, G>), dim3((unsigned)nb), dim3(kBlock), 0, s, U,
                       T, c.frag, c.ops, c.mesh, out, R, ra, rb, dt);
  else
    hipLaunchKernelGGL((k_stage_mfma<N, FORM, 1, G>), dim3((unsigned)nb), dim3(kBlock), 0, s, U,
                       T, c.frag, c.ops, c.mesh, out, R, ra, rb, dt);
  return hipGetLastError();
}

template <int N, int FORM>
hipError_t stage_staged_n(const dgpyr_ctx& c, int mode, const double* U, const double* T,
                          double* out, double* R, double ra, double rb, double dt, hipStream_t s) {
  const int64_t nb = (c.K + kEB - 1) / kEB;
  if (mode == 0)
    hipLaunchKernelGGL((k_stage_staged<N, FORM, 0>), dim3((unsigned)nb), dim3(kBlock), 0, s, U, T,
                       c.frag, c.ops, c.mesh, out, R, ra, rb, dt);
  else
    hipLaunchKernelGGL((k_stage_staged<N, FORM, 1>), dim3((unsigned)nb), dim3(kBlock), 0, s, U, T,
                       c.frag, c.ops, c.mesh, out, R, ra, rb, dt);
  return hipGetLastError();
}

template <int N>
hipError_t stage_mfma_dispatch(const dgpyr_ctx& c, int mode, const double* U, const double* T,
                               double* out, double* R, double ra, double rb, double dt,
                               hipStream_t s) {
  if (c.lds_operators) {
    if (c.precision == DGPYR_FP32_MFMA) {
      if constexpr (StagedDims<N, 1>::fits)
        return stage_staged_n<N, 1>(c, mode, U, T, out, R, ra, rb, dt, s);
    } else if constexpr (StagedDims<N, 0>::fits) {
      return stage_staged_n<N, 0>(c, mode, U, T, out, R, ra, rb, dt, s);
    }
  }
  const bool two = mfma_groups(c) == 2;
  if (c.precision == DGPYR_FP32_MFMA)
    return two ? stage_mfma_n<N, 1, 2>(c, mode, U, T, out, R, ra, rb, dt, s)
               : stage_mfma_n<N, 1, 1>(c, mode, U, T, out, R, ra, rb, dt, s);
  return two ? stage_mfma_n<N, 0, 2>(c, mode, U, T, out, R, ra, rb, dt, s)
             : stage_mfma_n<N, 0, 1>(c, mode, U, T, out, R, ra, rb, dt, s);
}

template <int N, int G>
hipError_t trace_mfma_g(const dgpyr_ctx& c, const double* U, double* T, hipStream_t s) {
  const int64_t nb = (c.K + kEB * G - 1) / (kEB * G);
  hipLaunchKernelGGL((k_trace_mfma<N, G>), dim3((unsigned)nb), dim3(kBlock), 0, s, U, T, c.frag,
                     c.K);
  return hipGetLastError();
}

template <int N>
hipError_t trace_mfma_n(const dgpyr_ctx& c, const double* U, double* T, hipStream_t s) {
  switch (trace_groups(c)) {
    case 4: return trace_mfma_g<N, 4>(c, U, T, s);
    case 2: return trace_mfma_g<N, 2>(c, U, T, s);
    default: return trace_mfma_g<N, 1>(c, U, T, s);
  }
}

template <int N, int FORM>
hipError_t surface_mfma_n(const dgpyr_ctx& c, int mode, const double* T, const double* vol,
                          double* out, double* R, double ra, double rb, double dt, hipStream_t s) {
  const int64_t nb = (c.K + kEB - 1) / kEB;
  if (mode == 0)
    hipLaunchKernelGGL((k_surface_mfma<N, FORM, 0>), dim3((unsigned)nb), dim3(kBlock), 0, s, T, vol,
                       c.frag, c.ops, c.mesh, out, R, ra, rb, dt);
  else
    hipLaunchKernelGGL((k_surface_mfma<N, FORM, 1>), dim3((unsigned)nb), dim3(kBlock), 0, s, T, vol,
                       c.frag, c.ops, c.mesh, out, R, ra, rb, dt);
  return hipGetLastError();
}

template <int N>
hipError_t surface_mfma_dispatch(const dgpyr_ctx& c, int mode, const double* T, const double* vol,
                                 double* out, double* R, double ra, double rb, double dt,
                                 hipStream_t s) {
  if (c.precision == DGPYR_FP32_MFMA) return surface_mfma_n<N, 1>(c, mode, T, vol, out, R, ra, rb, dt, s);
  return surface_mfma_n<N, 0>(c, mode, T, vol, out, R, ra, rb, dt, s);
}

template <int N, int FORM>
hipError_t volume_mfma_n(const dgpyr_ctx& c, const double* U, double* vol, hipStream_t s) {
  const int64_t nb = (c.K + kEB - 1) / kEB;
  hipLaunchKernelGGL((k_volume_mfma<N, FORM>), dim3((unsigned)nb), dim3(kBlock), 0, s, U, vol,
                     c.frag, c.ops, c.mesh);
  return hipGetLastError();
}

template <int N>
hipError_t volume_mfma_dispatch(const dgpyr_ctx& c, const double* U, double* vol, hipStream_t s) {
  if (c.precision == DGPYR_FP32_MFMA) return volume_mfma_n<N, 1>(c, U, vol, s);
  return volume_mfma_n<N, 0>(c, U, vol, s);
}

}  // namespace

#define DGPYR_DISPATCH_N(fn, ...)        \
  switch (c.N) {                         \
    case 0: return fn<0>(__VA_ARGS__);   \
    case 1: return fn<1>(__VA_ARGS__);   \
    case 2: return fn<2>(__VA_ARGS__);   \
    case 3: return fn<3>(__VA_ARGS__);   \
    case 4: return fn<4>(__VA_ARGS__);   \
    case 5: return fn<5>(__VA_ARGS__);   \
    case 6: return fn<6>(__VA_ARGS__);   \
    case 7: return fn<7>(__VA_ARGS__);   \
    case 8: return fn<8>(__VA_ARGS__);   \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_volume_mfma(const dgpyr_ctx& c, const double* U, double* vol, hipStream_t s) {
  DGPYR_DISPATCH_N(volume_mfma_dispatch, c, U, vol, s)
}

hipError_t launch_trace_mfma(const dgpyr_ctx& c, const double* U, double* T, hipStream_t s) {
  DGPYR_DISPATCH_N(trace_mfma_n, c, U, T, s)
}

hipError_t launch_stage_mfma(const dgpyr_ctx& c, int mode, const double* U, const double* T,
                             double* out, double* R, double ra, double rb, double dt,
                             hipStream_t s) {
  DGPYR_DISPATCH_N(stage_mfma_dispatch, c, mode, U, T, out, R, ra, rb, dt, s)
}

hipError_t launch_surface_mfma(const dgpyr_ctx& c, int mode, const double* T, const double* vol,
                               double* out, double* R, double ra, double rb, double dt,
                               hipStream_t s) {
  DGPYR_DISPATCH_N(surface_mfma_dispatch, c, mode, T, vol, out, R, ra, rb, dt, s)
}

}  // namespace dgpyr
