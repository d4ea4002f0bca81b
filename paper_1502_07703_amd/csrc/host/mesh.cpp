// Per-element geometry checks and topological face matching.
#include "mesh.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>

#include "dgpyr.h"
#include "../geom.hpp"

namespace dgpyr {

namespace {

inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Vertices of each face in parametrisation order.
//   quad (face 0): corner at (a,b) = (-1,-1), (1,-1), (1,1), (-1,1)
//   triangles: edge start (sigma = -1), edge end (sigma = +1), apex
const int kQuad[4] = {0, 1, 2, 3};
const int kTri[4][3] = {{0, 3, 4}, {1, 2, 4}, {0, 1, 4}, {3, 2, 4}};

struct FaceKey {
  std::array<int64_t, 4> v;  // sorted vertex ids, triangles padded with -1
  int64_t slot;              // 5 * elem + face
  bool operator<(const FaceKey& o) const {
    if (v != o.v) return v < o.v;
    return slot < o.slot;
  }
};

// Corner index of (a, b) in {-1, 1}^2 in the quad order above.
inline int corner_of(int a, int b) {
  if (b < 0) return a < 0 ? 0 : 1;
  return a > 0 ? 2 : 3;
}

}  // namespace

namespace {

// Lowest element in [e_lo, e_hi) containing point xs (bounding box, then
// Newton on x(a,b,c) = (1-c)/2 B(a,b) + (1+c)/2 x4 from the element middle);
// returns the element or -1 and the collapsed coordinates in abc.
int64_t find_point(const double* verts, const double* xs, int64_t e_lo, int64_t e_hi, double* abc) {
  for (int64_t e = e_lo; e < e_hi; ++e) {
    const double* x = verts + (size_t)e * 16;
    bool inbox = true;
    for (int d = 0; d < 3 && inbox; ++d) {
      double lo = x[d], hi = x[d];
      for (int v = 1; v < 5; ++v) {
        lo = std::min(lo, x[3 * v + d]);
        hi = std::max(hi, x[3 * v + d]);
      }
      const double pad = 1e-9 * std::max(1.0, hi - lo);
      inbox = xs[d] >= lo - pad && xs[d] <= hi + pad;
    }
    if (!inbox) continue;
    double a = 0.0, b = 0.0, c = -0.5;
    bool ok = false, polish = false;
    for (int it = 0; it < 60; ++it) {
      double B[3], Ba[3], Bb[3], F[3], G[9];
      for (int d = 0; d < 3; ++d) {
        const double x0 = x[d], x1 = x[3 + d], x2 = x[6 + d], x3 = x[9 + d], x4 = x[12 + d];
        B[d] = 0.25 * ((1 - a) * (1 - b) * x0 + (1 + a) * (1 - b) * x1 + (1 + a) * (1 + b) * x2 +
                       (1 - a) * (1 + b) * x3);
        Ba[d] = 0.25 * ((1 - b) * (x1 - x0) + (1 + b) * (x2 - x3));
        Bb[d] = 0.25 * ((1 - a) * (x3 - x0) + (1 + a) * (x2 - x1));
        F[d] = 0.5 * (1 - c) * B[d] + 0.5 * (1 + c) * x4 - xs[d];
        G[3 * d + 0] = 0.5 * (1 - c) * Ba[d];
        G[3 * d + 1] = 0.5 * (1 - c) * Bb[d];
        G[3 * d + 2] = 0.5 * (x4 - B[d]);
      }
      // solve G delta = -F by Cramer's rule
      const double det = G[0] * (G[4] * G[8] - G[5] * G[7]) - G[1] * (G[3] * G[8] - G[5] * G[6]) +
                         G[2] * (G[3] * G[7] - G[4] * G[6]);
      if (!(std::fabs(det) > 0)) break;
      double dl[3];
      for (int k = 0; k < 3; ++k) {
        double M[9];
        for (int i = 0; i < 9; ++i) M[i] = G[i];
        for (int r = 0; r < 3; ++r) M[3 * r + k] = -F[r];
        dl[k] = (M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                 M[2] * (M[3] * M[7] - M[4] * M[6])) / det;
      }
      a += dl[0];
      b += dl[1];
      c += dl[2];
      if (std::fabs(a) > 10 || std::fabs(b) > 10 || std::fabs(c) > 10) break;
      // Steps stall at a few ulps of O(1) coordinates (more where the map
      // is ill-conditioned); a step below 1e-12 has converged, and one more
      // step polishes the root to rounding.
      if (polish) {
        ok = true;
        break;
      }
      if (std::fabs(dl[0]) + std::fabs(dl[1]) + std::fabs(dl[2]) < 1e-12) polish = true;
    }
    const double sl = 1e-10;
    if (ok && a >= -1 - sl && a <= 1 + sl && b >= -1 - sl && b <= 1 + sl && c >= -1 - sl &&
        c <= 1 + sl) {
      abc[0] = a;
      abc[1] = b;
      abc[2] = c;
      return e;
    }
  }
  return -1;
}

}  // namespace

int locate_sources(const RefOps& ops, int nsrc, const double* src, const int64_t* range,
                   MeshData& md, std::string& err) {
  char buf[256];
  md.nsrc = nsrc;
  md.src_of.assign((size_t)md.K, -1);
  md.src_phi.assign((size_t)nsrc * ops.Np, 0.0);
  md.src_par.assign((size_t)nsrc * 4, 0.0);
  md.src_elem.assign((size_t)nsrc, -1);
  md.src_abc.assign((size_t)nsrc * 3, 0.0);
  for (int s = 0; s < nsrc; ++s) {
    const double* xs = src + 6 * s;
    const int64_t e_lo = range ? range[2 * s] : 0, e_hi = range ? range[2 * s + 1] : md.K;
    double abc[3];
    const int64_t found = find_point(md.verts.data(), xs, e_lo, e_hi, abc);
    if (found < 0) {
      std::snprintf(buf, sizeof buf, "source %d at (%g, %g, %g) lies in no element", s, xs[0],
                    xs[1], xs[2]);
      err = buf;
      return DGPYR_E_ARG;
    }
    if (md.src_of[(size_t)found] >= 0) {
      std::snprintf(buf, sizeof buf, "sources %d and %d lie in the same element", md.src_of[found], s);
      err = buf;
      return DGPYR_E_UNSUPPORTED;
    }
    md.src_of[(size_t)found] = s;
    md.src_elem[(size_t)s] = found;
    for (int k = 0; k < 3; ++k) md.src_abc[(size_t)3 * s + k] = abc[k];
    eval_basis(ops.N, abc[0], abc[1], abc[2], &md.src_phi[(size_t)s * ops.Np]);
    md.src_par[4 * s + 0] = xs[3];
    md.src_par[4 * s + 1] = xs[4];
    md.src_par[4 * s + 2] = xs[5] > 0 ? xs[5] : 1.0 / xs[4];
  }
  return 0;
}

int locate_receivers(const RefOps& ops, int nrec, const double* xyz, const double* verts,
                     int64_t K, std::vector<int64_t>& elem, std::vector<double>& phi,
                     std::string& err) {
  elem.assign((size_t)nrec, -1);
  phi.assign((size_t)nrec * ops.Np, 0.0);
  for (int r = 0; r < nrec; ++r) {
    double abc[3];
    const int64_t e = find_point(verts, xyz + 3 * r, 0, K, abc);
    if (e < 0) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "receiver %d at (%g, %g, %g) lies in no element", r,
                    xyz[3 * r], xyz[3 * r + 1], xyz[3 * r + 2]);
      err = buf;
      return DGPYR_E_ARG;
    }
    elem[(size_t)r] = e;
    eval_basis(ops.N, abc[0], abc[1], abc[2], &phi[(size_t)r * ops.Np]);
  }
  return 0;
}

int build_mesh(const RefOps& ops, int64_t nverts, const double* xyz, int64_t nelems,
               const int64_t* e2v_geom, const double* rho, const double* kappa, MeshData& md,
               std::string& err, const int64_t* pair_ids) {
  const int64_t* e2v = e2v_geom;
  char buf[256];
  const int64_t K = nelems;
  md.K = K;
  md.verts.assign((size_t)K * 16, 0.0);
  md.conn.assign((size_t)K * 8, -1);
  md.mat.assign((size_t)K * 4, 0.0);

  for (int64_t e = 0; e < K; ++e)
    for (int i = 0; i < 5; ++i) {
      const int64_t v = e2v[5 * e + i];
      if (v < 0 || v >= nverts) {
        std::snprintf(buf, sizeof buf, "element %lld: vertex index %lld out of range",
                      (long long)e, (long long)v);
        err = buf;
        return DGPYR_E_ARG;
      }
      for (int d = 0; d < 3; ++d) md.verts[(size_t)e * 16 + 3 * i + d] = xyz[3 * v + d];
    }

  // Geometry: J > 0 at the four base corners implies J > 0 everywhere, since J
  // is bilinear in (a, b) and constant in c (Lemma 1).  Also |dK| / |K|.
  const int n1 = ops.Nq1;
  md.inv_length_max = 0.0;
  md.inv_length.assign((size_t)K, 0.0);
  for (int64_t e = 0; e < K; ++e) {
    const double* x = &md.verts[(size_t)e * 16];
    const double r = rho ? rho[e] : 1.0;
    const double k = kappa ? kappa[e] : 1.0;
    if (!(r > 0) || !(k > 0)) {
      std::snprintf(buf, sizeof buf, "element %lld: rho and kappa must be positive", (long long)e);
      err = buf;
      return DGPYR_E_ARG;
    }
    md.mat[4 * e + 0] = k;
    md.mat[4 * e + 1] = 1.0 / r;
    md.mat[4 * e + 2] = std::sqrt(k / r) * r;
    md.mat[4 * e + 3] = 1.0;  // time-step scale (per-problem dt in batches)
    double adj[9], J;
    for (int ca = -1; ca <= 1; ca += 2)
      for (int cb = -1; cb <= 1; cb += 2) {
        pyr_metric(x, ca, cb, adj, &J);
        if (!(J > 0)) {
          std::snprintf(buf, sizeof buf,
                        "element %lld: Jacobian %.3e <= 0 at base corner (%d,%d); check the "
                        "vertex order (base counter-clockwise seen from the apex)",
                        (long long)e, J, ca, cb);
          err = buf;
          return DGPYR_E_MESH;
        }
      }
    // volume = sum_q w_q J(a_q, b_q); J does not depend on c
    double vol = 0.0;
    for (int m = 0; m < n1; ++m)
      for (int p = 0; p < n1; ++p) {
        pyr_metric(x, ops.xg[p], ops.xg[m], adj, &J);
        vol += ops.wg[p] * ops.wg[m] * J * (8.0 / 3.0) / 4.0;
      }
    // surface area |dK|: the base with the face rule (as the flux integrals
    // are taken), the planar triangles in closed form
    double area = 0.0;
    for (int m = 0; m < n1; ++m)
      for (int p = 0; p < n1; ++p) {
        double nrm[3];
        pyr_face_normal(x, 0, ops.xg[p], ops.xg[m], nrm);
        area += ops.wg[p] * ops.wg[m] * std::sqrt(dot3(nrm, nrm));
      }
    for (int f = 1; f < 5; ++f) {
      double nrm[3];
      pyr_face_normal(x, f, 0.0, 0.0, nrm);
      area += 2.0 * std::sqrt(dot3(nrm, nrm));  // parameter-space area of a triangle is 2
    }
    md.inv_length[(size_t)e] = std::sqrt(k / r) * area / vol;
    md.inv_length_max = std::max(md.inv_length_max, md.inv_length[(size_t)e]);
  }

  // Faces: sort by vertex set (vertex identities when given), pair equal keys.
  std::vector<int64_t> paired;
  if (pair_ids) {
    for (int64_t v = 0; v < nverts; ++v)
      if (pair_ids[v] < 0 || pair_ids[v] >= nverts) {
        std::snprintf(buf, sizeof buf, "pair id of vertex %lld out of range", (long long)v);
        err = buf;
        return DGPYR_E_ARG;
      }
    paired.resize((size_t)K * 5);
    for (size_t i = 0; i < paired.size(); ++i) paired[i] = pair_ids[e2v_geom[i]];
    e2v = paired.data();
  }
  std::vector<FaceKey> keys((size_t)K * 5);
  for (int64_t e = 0; e < K; ++e) {
    const int64_t* ev = &e2v[5 * e];
    for (int f = 0; f < 5; ++f) {
      FaceKey& fk = keys[(size_t)e * 5 + f];
      fk.slot = 5 * e + f;
      if (f == 0) {
        for (int i = 0; i < 4; ++i) fk.v[i] = ev[kQuad[i]];
      } else {
        for (int i = 0; i < 3; ++i) fk.v[i] = ev[kTri[f - 1][i]];
        fk.v[3] = -1;
      }
      std::sort(fk.v.begin(), fk.v.end());
      for (int i = 1; i < 4; ++i)
        if (fk.v[i] >= 0 && fk.v[i] == fk.v[i - 1]) {
          std::snprintf(buf, sizeof buf, "element %lld face %d has a repeated vertex",
                        (long long)e, f);
          err = buf;
          return DGPYR_E_MESH;
        }
    }
  }
  std::sort(keys.begin(), keys.end());
  std::vector<uint32_t> code((size_t)K, 0u);
  const size_t F = keys.size();
  size_t i = 0;
  while (i < F) {
    size_t j = i + 1;
    while (j < F && keys[j].v == keys[i].v) ++j;
    if (j - i > 2) {
      std::snprintf(buf, sizeof buf, "a face of element %lld is shared by %zu elements",
                    (long long)(keys[i].slot / 5), j - i);
      err = buf;
      return DGPYR_E_NONCONFORMING;
    }
    if (j - i == 2) {
      for (int side = 0; side < 2; ++side) {
        const int64_t s0 = keys[i + side].slot, s1 = keys[i + 1 - side].slot;
        const int64_t e0 = s0 / 5, e1 = s1 / 5;
        const int f0 = (int)(s0 % 5), f1 = (int)(s1 % 5);
        const int64_t* v0 = &e2v[5 * e0];
        const int64_t* v1 = &e2v[5 * e1];
        int orient = -1;
        if (f0 == 0) {
          if (f1 != 0) { orient = -1; }
          else {
            for (int o = 0; o < 8 && orient < 0; ++o) {
              bool ok = true;
              for (int ca = -1; ca <= 1 && ok; ca += 2)
                for (int cb = -1; cb <= 1 && ok; cb += 2) {
                  const bool swap = (o >> 2) & 1;
                  int X = swap ? cb : ca, Y = swap ? ca : cb;
                  if (o & 1) X = -X;
                  if ((o >> 1) & 1) Y = -Y;
                  ok = v0[kQuad[corner_of(ca, cb)]] == v1[kQuad[corner_of(X, Y)]];
                }
              if (ok) orient = o;
            }
          }
        } else if (f1 != 0) {
          const int* t0 = kTri[f0 - 1];
          const int* t1 = kTri[f1 - 1];
          if (v0[t0[2]] == v1[t1[2]]) {
            if (v0[t0[0]] == v1[t1[0]] && v0[t0[1]] == v1[t1[1]]) orient = 0;
            else if (v0[t0[0]] == v1[t1[1]] && v0[t0[1]] == v1[t1[0]]) orient = 1;
          }
        }
        if (orient < 0) {
          std::snprintf(buf, sizeof buf,
                        "elements %lld and %lld share face vertices but their face "
                        "parametrisations do not match (different face types or apexes)",
                        (long long)e0, (long long)e1);
          err = buf;
          return DGPYR_E_NONCONFORMING;
        }
        md.conn[(size_t)e0 * 8 + f0] = (int32_t)e1;
        code[e0] |= (uint32_t)(f1 | (orient << 3)) << (6 * f0);
      }
    }
    i = j;
  }
  for (int64_t e = 0; e < K; ++e) md.conn[(size_t)e * 8 + 5] = (int32_t)code[e];

  // Groups of 6 consecutive elements sharing an apex whose triangle faces all
  // pair inside the group (pyramids from splitting a hexahedron).
  md.hex_groups = (K % 6 == 0) && K > 0;
  for (int64_t g = 0; md.hex_groups && g < K / 6; ++g)
    for (int64_t e = 6 * g; e < 6 * g + 6 && md.hex_groups; ++e) {
      if (e2v[5 * e + 4] != e2v[5 * 6 * g + 4]) md.hex_groups = false;
      for (int f = 1; f < 5; ++f) {
        const int32_t nb = md.conn[(size_t)e * 8 + f];
        if (nb < 6 * g || nb >= 6 * g + 6) md.hex_groups = false;
      }
    }
  return 0;
}

}  // namespace dgpyr
