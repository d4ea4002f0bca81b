// Initial data and error evaluation on the volume cubature: physical points
// and weights, L2 projection, and evaluation of a state at the points.
// Not on the per-stage path; plain FP64 vector-ALU kernels.
#include <hip/hip_runtime.h>

#include "context.hpp"
#include "geom.hpp"

namespace dgpyr {
namespace {

constexpr int kThreads = 256;

// Physical coordinates x(a, b, c) = (1-c)/2 B(a, b) + (1+c)/2 x4 of every
// volume cubature point and, optionally, the weight w_q J(a_q, b_q).
__global__ void k_points(DevOps ops, DevMesh mesh, int n1, int Nc, const double* __restrict__ xc,
                         double* __restrict__ xyz, double* __restrict__ wJ) {
  const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (gid >= mesh.K * Nc) return;
  const int64_t e = gid / Nc;
  const int q = (int)(gid - e * Nc);
  const int p = q % n1, m = (q / n1) % n1, r = q / (n1 * n1);
  const double a = ops.xg[p], b = ops.xg[m], c = xc[r];
  const double* x = mesh.verts + e * 16;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double B = 0.25 * ((1 - a) * (1 - b) * x[d] + (1 + a) * (1 - b) * x[3 + d] +
                             (1 + a) * (1 + b) * x[6 + d] + (1 - a) * (1 + b) * x[9 + d]);
    xyz[gid * 3 + d] = 0.5 * (1 - c) * B + 0.5 * (1 + c) * x[12 + d];
  }
  if (wJ) wJ[gid] = ops.wv[q] * pyr_jac(x, a, b);
}

// U_i = sum_q w_q J_q phi_i(q) f_q / M_ii (M diagonal, Lemma 3), per field.
__global__ void k_project(DevOps ops, DevMesh mesh, int Np, int Nc, int n1, int nf,
                          const double* __restrict__ f, double* __restrict__ U) {
  const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (gid >= mesh.K * nf * Np) return;
  const int64_t e = gid / (nf * Np);
  const int rem = (int)(gid - e * nf * Np);
  const int fld = rem / Np, i = rem - fld * Np;
  const double* x = mesh.verts + e * 16;
  const double* fe = f + (e * nf + fld) * Nc;
  double acc = 0.0;
  for (int q = 0; q < Nc; ++q) {
    const int p = q % n1, m = (q / n1) % n1;
    acc += ops.wv[q] * pyr_jac(x, ops.xg[p], ops.xg[m]) * ops.V[(int64_t)q * Np + i] * fe[q];
  }
  U[gid] = acc / (pyr_jac(x, ops.na[i], ops.nb[i]) * ops.wwc[i]);
}

// f_q = sum_n phi_n(q) U_n per field.
__global__ void k_eval(DevOps ops, int64_t K, int Np, int Nc, int nf, const double* __restrict__ U,
                       double* __restrict__ f) {
  const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (gid >= K * nf * Nc) return;
  const int64_t ef = gid / Nc;
  const int q = (int)(gid - ef * Nc);
  const double* u = U + ef * Np;
  double acc = 0.0;
  for (int n = 0; n < Np; ++n) acc += ops.V[(int64_t)q * Np + n] * u[n];
  f[gid] = acc;
}

// Step counter used for source times: set or advance by one (one thread).
__global__ void k_clock(double* clock, double value, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) clock[0] = add ? clock[0] + value : value;
}

// x[0 .. n) = value, grid-stride (a kernel rather than a memset node, so the
// call is safe inside captured graphs).
__global__ void k_fill(double* __restrict__ x, int64_t n, double value) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    x[i] = value;
}

// Watchdog: if any of x[0 .. n) is a NaN or an infinity (all exponent bits
// set), lower *first_bad to step.  The minimum does not depend on the order of
// the updates, so the outcome is deterministic; x is only read.
__global__ void k_nonfinite(const double* __restrict__ x, int64_t n, unsigned long long step,
                            unsigned long long* first_bad) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    bad |= ((__double_as_longlong(x[i]) >> 52) & 0x7ff) == 0x7ff;
  if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicMin(first_bad, step);
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

hipError_t launch_fill(double* x, int64_t n, double value, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)(nb < 65536 ? nb : 65536)), dim3(kThreads), 0, s, x, n,
                     value);
  return hipGetLastError();
}

hipError_t launch_nonfinite(const double* x, int64_t n, unsigned long long step,
                            unsigned long long* first_bad, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(kThreads), 0, s,
                     x, n, step, first_bad);
  return hipGetLastError();
}

hipError_t launch_clock(double* clock, double value, bool add, hipStream_t s) {
  hipLaunchKernelGGL(k_clock, dim3(1), dim3(64), 0, s, clock, value, add ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_points(const dgpyr_ctx& c, double* xyz, double* wJ, hipStream_t s) {
  hipLaunchKernelGGL(k_points, dim3(nblocks(c.K * c.Nc)), dim3(kThreads), 0, s, c.ops, c.mesh,
                     c.N + 1, c.Nc, c.xc, xyz, wJ);
  return hipGetLastError();
}

hipError_t launch_project(const dgpyr_ctx& c, const double* f, double* U, hipStream_t s) {
  hipLaunchKernelGGL(k_project, dim3(nblocks(c.K * c.nfields * c.Np)), dim3(kThreads), 0, s, c.ops,
                     c.mesh, c.Np, c.Nc, c.N + 1, c.nfields, f, U);
  return hipGetLastError();
}

hipError_t launch_eval(const dgpyr_ctx& c, const double* U, double* f, hipStream_t s) {
  hipLaunchKernelGGL(k_eval, dim3(nblocks(c.K * c.nfields * c.Nc)), dim3(kThreads), 0, s, c.ops, c.K,
                     c.Np, c.Nc, c.nfields, U, f);
  return hipGetLastError();
}

}  // namespace dgpyr
