// Penalty flux of the acoustic DG scheme at one face point (Section 4.3).
#pragma once

#include <hip/hip_runtime.h>

#include "context.hpp"
#include "geom.hpp"

namespace dgpyr {

// Traces at one face point: the element's own (pm, um) and, on a face with a
// neighbour, the neighbour's at the matching point (pp, up) with its rho c.
struct FaceTraces {
  double pm, um0, um1, um2;
  double pp, up0, up1, up2, zp;
  bool inner;
};

// Weighted flux from the traces at one face point, given the point's unit
// outward normal n = (n0, n1, n2), w = face weight x surface Jacobian sJ and
// the element's rho c zm.  A face without a neighbour gets the mirror state.
// With [[a]] = a+ - a-, tau_p = alpha / {rho c}, tau_u = alpha {rho c}:
//   F[0]   = w (n.[[u]] - tau_p [[p]]) / 2
//   F[1+k] = w n_k ([[p]] - tau_u n.[[u]]) / 2
__device__ __forceinline__ void flux_from_traces(const FaceTraces& t, const DevMesh& mesh,
                                                 double zm, double n0, double n1, double n2,
                                                 double w, double F[4]) {
  double pp, up0, up1, up2, zp;
  if (t.inner) {
    pp = t.pp; up0 = t.up0; up1 = t.up1; up2 = t.up2;
    zp = t.zp;
  } else {
    const double un = n0 * t.um0 + n1 * t.um1 + n2 * t.um2;
    if (mesh.bc == DGPYR_BC_WALL) {
      pp = t.pm; up0 = t.um0 - 2 * un * n0; up1 = t.um1 - 2 * un * n1; up2 = t.um2 - 2 * un * n2;
    } else {
      pp = -t.pm; up0 = t.um0; up1 = t.um1; up2 = t.um2;
    }
    zp = zm;
  }
  const double zavg = 0.5 * (zm + zp);
  const double taup = mesh.alpha / zavg, tauu = mesh.alpha * zavg;
  const double jp = pp - t.pm;
  const double jun = n0 * (up0 - t.um0) + n1 * (up1 - t.um1) + n2 * (up2 - t.um2);
  const double Pu = 0.5 * w * (jp - tauu * jun);
  F[0] = 0.5 * w * (jun - taup * jp);
  F[1] = n0 * Pu;
  F[2] = n1 * Pu;
  F[3] = n2 * Pu;
}

// Weighted flux at face point q (face f = q / Nfq) of element e, given the
// point's unit outward normal and surface Jacobian sJ: the element's own
// trace and the neighbour's are read from T ([K][Nfc][4]) through the
// connectivity code.
template <int Nfq>
__device__ __forceinline__ void face_flux_at(const double* __restrict__ T, const DevOps& ops,
                                             const DevMesh& mesh, int64_t e, int q, double n0,
                                             double n1, double n2, double sJ, double F[4]) {
  constexpr int Nfc = 5 * Nfq;
  const int f = q / Nfq, qq = q - f * Nfq;
  const double* tm = T + (e * Nfc + q) * 4;
  FaceTraces t;
  t.pm = tm[0]; t.um0 = tm[1]; t.um1 = tm[2]; t.um2 = tm[3];
  const int nb = mesh.conn[e * 8 + f];
  t.inner = nb >= 0;
  if (t.inner) {
    const int code = (mesh.conn[e * 8 + 5] >> (6 * f)) & 63;
    const int nf = code & 7, o = code >> 3;
    const int pi = ops.perm[(f == 0 ? o : 8 + o) * Nfq + qq];
    const double* tp = T + ((int64_t)nb * Nfc + nf * Nfq + pi) * 4;
    t.pp = tp[0]; t.up0 = tp[1]; t.up1 = tp[2]; t.up2 = tp[3];
    t.zp = mesh.mat[(int64_t)nb * 4 + 2];
  }
  flux_from_traces(t, mesh, mesh.mat[e * 4 + 2], n0, n1, n2, ops.wf[q] * sJ, F);
}

// Unit outward normal and surface Jacobian at face point q of an element
// with vertices x: nrm = (N / |N|, |N|) for the area-weighted normal N.
__device__ __forceinline__ void face_normal_unit(const double* x, int f, double a, double b,
                                                 double nrm[4]) {
  double Nv[3];
  pyr_face_normal(x, f, a, b, Nv);
  const double sJ = sqrt(Nv[0] * Nv[0] + Nv[1] * Nv[1] + Nv[2] * Nv[2]);
  nrm[0] = Nv[0] / sJ;
  nrm[1] = Nv[1] / sJ;
  nrm[2] = Nv[2] / sJ;
  nrm[3] = sJ;
}

// face_flux_at with the normal computed from the element's vertices x.
template <int Nfq>
__device__ __forceinline__ void face_flux(const double* __restrict__ T, const DevOps& ops,
                                          const DevMesh& mesh, const double* x, int64_t e, int q,
                                          double F[4]) {
  double nrm[4];
  face_normal_unit(x, q / Nfq, ops.fa[q], ops.fb[q], nrm);
  face_flux_at<Nfq>(T, ops, mesh, e, q, nrm[0], nrm[1], nrm[2], nrm[3], F);
}

// Ricker wavelet (1 - 2 a) exp(-a), a = (pi f0 (t - delay))^2.
__device__ __forceinline__ double ricker_wavelet(double t, double f0, double delay) {
  const double x = 3.14159265358979323846 * f0 * (t - delay);
  const double a = x * x;
  return (1.0 - 2.0 * a) * exp(-a);
}

// Point-source contribution b_i = amp R(t) phi_i(xi_s) to the pressure
// coefficient i of element e (zero for elements without a source).
template <int Np>
__device__ __forceinline__ double source_term(const DevMesh& mesh, int64_t e, int i) {
  if (!mesh.src_of) return 0.0;
  const int s = mesh.src_of[e];
  if (s < 0) return 0.0;
  const double* par = mesh.src_par + 4 * s;
  const double n = mesh.clock ? mesh.clock[0] : 0.0;
  const double t = mesh.t_base + (n + mesh.c_stage) * mesh.dt_time * mesh.mat[e * 4 + 3];
  return par[0] * ricker_wavelet(t, par[1], par[2]) * mesh.src_phi[(int64_t)s * Np + i];
}

// Inverse mass, material scaling and output of one coefficient (Algorithm 3):
// rhs_p = -kappa acc_p / M_ii, rhs_u = -(1/rho) acc_u / M_ii with the diagonal
// M_ii = J(a_i, b_i) w_i w_j 2/(2k+3) of Lemma 3.  MODE 0 writes rhs; MODE 1
// performs R <- ra R + dt rhs (R not read when ra == 0), U <- U + rb R.
template <int MODE>
__device__ __forceinline__ void finish_coeff(double acc, double minv, double mat, double* out,
                                             double* R, int64_t idx, double ra, double rb,
                                             double dt) {
  const double rhs = -mat * minv * acc;
  if (MODE == 0) {
    out[idx] = rhs;
  } else {
    const double rn = (ra == 0.0 ? 0.0 : ra * R[idx]) + dt * rhs;
    R[idx] = rn;
    out[idx] += rb * rn;
  }
}

}  // namespace dgpyr
