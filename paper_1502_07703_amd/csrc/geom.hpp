// Vertex-map geometry shared by the host builders and the device kernels.
//
// Section 2: the vertex map built from Bedrosian's vertex functions equals, in
// collapsed coordinates, x(a, b, c) = (1-c)/2 B(a, b) + (1+c)/2 x4 with
//   B(a,b) = 1/4 [(1-a)(1-b) x0 + (1+a)(1-b) x1 + (1+a)(1+b) x2 + (1-a)(1+b) x3].
// Its Jacobian matrix has columns
//   x_r = B_a,  x_s = B_b,  x_t = (x4 - B)/2 + (1+a)/2 B_a + (1+b)/2 B_b,
// which depend on (a, b) only; J = det is bilinear in (a, b) (Lemma 1).
#pragma once

#include <hip/hip_runtime.h>

namespace dgpyr {

// x: 15 doubles (x0..x4).  adj[3*rho + d] = J * d rho / d x_d (rows of the
// cofactor matrix: x_s x x_t, x_t x x_r, x_r x x_s), *J = det.
__host__ __device__ inline void pyr_metric(const double* x, double a, double b, double* adj, double* J) {
  double Ba[3], Bb[3], xt[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double x0 = x[d], x1 = x[3 + d], x2 = x[6 + d], x3 = x[9 + d], x4 = x[12 + d];
    const double B = 0.25 * ((1 - a) * (1 - b) * x0 + (1 + a) * (1 - b) * x1 +
                             (1 + a) * (1 + b) * x2 + (1 - a) * (1 + b) * x3);
    Ba[d] = 0.25 * ((1 - b) * (x1 - x0) + (1 + b) * (x2 - x3));
    Bb[d] = 0.25 * ((1 - a) * (x3 - x0) + (1 + a) * (x2 - x1));
    xt[d] = 0.5 * (x4 - B) + 0.5 * (1 + a) * Ba[d] + 0.5 * (1 + b) * Bb[d];
  }
  adj[0] = Bb[1] * xt[2] - Bb[2] * xt[1];
  adj[1] = Bb[2] * xt[0] - Bb[0] * xt[2];
  adj[2] = Bb[0] * xt[1] - Bb[1] * xt[0];
  adj[3] = xt[1] * Ba[2] - xt[2] * Ba[1];
  adj[4] = xt[2] * Ba[0] - xt[0] * Ba[2];
  adj[5] = xt[0] * Ba[1] - xt[1] * Ba[0];
  adj[6] = Ba[1] * Bb[2] - Ba[2] * Bb[1];
  adj[7] = Ba[2] * Bb[0] - Ba[0] * Bb[2];
  adj[8] = Ba[0] * Bb[1] - Ba[1] * Bb[0];
  *J = Ba[0] * adj[0] + Ba[1] * adj[1] + Ba[2] * adj[2];
}

// Jacobian determinant only.
__host__ __device__ inline double pyr_jac(const double* x, double a, double b) {
  double adj[9], J;
  pyr_metric(x, a, b, adj, &J);
  return J;
}

// J(a, b) is bilinear (Lemma 1): with B = P + a Q + b S + ab W and D = x4 - P,
//   J = [B_a, B_b, (x4 - B)/2] = ([Q,S,D] + a [Q,W,D] + b [W,S,D] + ab [Q,S,W]) / 2,
// [u,v,w] = (u x v).w (the (1+a)/2 B_a and (1+b)/2 B_b parts of x_t drop out of
// the determinant, and the a^2, b^2 terms cancel).  c[4] = coefficients of
// 1, a, b, ab.
__host__ __device__ inline void pyr_jac_coeffs(const double* x, double* c) {
  double P[3], Q[3], S[3], W[3], D[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double x0 = x[d], x1 = x[3 + d], x2 = x[6 + d], x3 = x[9 + d];
    P[d] = 0.25 * (x0 + x1 + x2 + x3);
    Q[d] = 0.25 * (-x0 + x1 + x2 - x3);
    S[d] = 0.25 * (-x0 - x1 + x2 + x3);
    W[d] = 0.25 * (x0 - x1 + x2 - x3);
    D[d] = x[12 + d] - P[d];
  }
  const double qs0 = Q[1] * S[2] - Q[2] * S[1], qs1 = Q[2] * S[0] - Q[0] * S[2],
               qs2 = Q[0] * S[1] - Q[1] * S[0];
  const double qw0 = Q[1] * W[2] - Q[2] * W[1], qw1 = Q[2] * W[0] - Q[0] * W[2],
               qw2 = Q[0] * W[1] - Q[1] * W[0];
  const double ws0 = W[1] * S[2] - W[2] * S[1], ws1 = W[2] * S[0] - W[0] * S[2],
               ws2 = W[0] * S[1] - W[1] * S[0];
  c[0] = 0.5 * (qs0 * D[0] + qs1 * D[1] + qs2 * D[2]);
  c[1] = 0.5 * (qw0 * D[0] + qw1 * D[1] + qw2 * D[2]);
  c[2] = 0.5 * (ws0 * D[0] + ws1 * D[1] + ws2 * D[2]);
  c[3] = 0.5 * (qs0 * W[0] + qs1 * W[1] + qs2 * W[2]);
}

__host__ __device__ inline double pyr_jac_eval(const double* c, double a, double b) {
  return c[0] + a * c[1] + b * (c[2] + a * c[3]);
}

// Outward area-weighted normal N (|N| = surface Jacobian of the face
// parametrisation) on face f at collapsed (a, b):
//   base (c = -1):      N = -B_a x B_b                      (varies with a, b)
//   a = -1:             N = -(x3 - x0) x (x4 - x0) / 4      (planar, constant)
//   a = +1:             N =  (x2 - x1) x (x4 - x1) / 4
//   b = -1:             N =  (x1 - x0) x (x4 - x0) / 4
//   b = +1:             N = -(x2 - x3) x (x4 - x3) / 4
// On the triangles the factor (1-c)/2 of the collapsed parametrisation is
// carried by the Gauss-Jacobi(1,0) weight.
__host__ __device__ inline void pyr_face_normal(const double* x, int f, double a, double b, double* N) {
  double u[3], v[3], s;
  if (f == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      u[d] = 0.25 * ((1 - b) * (x[3 + d] - x[d]) + (1 + b) * (x[6 + d] - x[9 + d]));
      v[d] = 0.25 * ((1 - a) * (x[9 + d] - x[d]) + (1 + a) * (x[6 + d] - x[3 + d]));
    }
    s = -1.0;
  } else {
    int o, p, q;
    if (f == 1) { o = 0; p = 3; q = 4; s = -0.25; }
    else if (f == 2) { o = 1; p = 2; q = 4; s = 0.25; }
    else if (f == 3) { o = 0; p = 1; q = 4; s = 0.25; }
    else { o = 3; p = 2; q = 4; s = -0.25; }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      u[d] = x[3 * p + d] - x[3 * o + d];
      v[d] = x[3 * q + d] - x[3 * o + d];
    }
  }
  N[0] = s * (u[1] * v[2] - u[2] * v[1]);
  N[1] = s * (u[2] * v[0] - u[0] * v[2]);
  N[2] = s * (u[0] * v[1] - u[1] * v[0]);
}

}  // namespace dgpyr
