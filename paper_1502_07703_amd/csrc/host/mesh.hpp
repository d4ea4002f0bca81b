// Host-side per-element geometry and face connectivity.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "refops.hpp"

namespace dgpyr {

// Per-element data handed to the device.
//   verts  [K][16]: x0..x4 (15 doubles) and one pad.
//   conn   [K][8] int32: neighbour element of faces 0..4 (-1 on the boundary),
//          then one packed word: for face f, bits 6f..6f+2 hold the
//          neighbour's face id and bits 6f+3..6f+5 the orientation code
//          (quad: 0..7 as in quad_perm, triangle: 0..1 as in tri_perm).
//   mat    [K][4]: kappa, 1/rho, rho*c, time-step scale (1 for one problem).
struct MeshData {
  int64_t K = 0;
  std::vector<double> verts;
  std::vector<int32_t> conn;
  std::vector<double> mat;
  double inv_length_max = 0.0;  // max_K c_K |dK| / |K|
  std::vector<double> inv_length;  // [K] c_K |dK| / |K|
  bool hex_groups = false;
  // point sources: src_of [K] (-1 = none), src_phi [nsrc][Np], src_par [nsrc][4]
  std::vector<int32_t> src_of;
  std::vector<double> src_phi, src_par;
  std::vector<int64_t> src_elem;  // [nsrc] containing element
  std::vector<double> src_abc;    // [nsrc][3] collapsed coordinates there
  int nsrc = 0;
};

// Locates each source point (x, y, z, amplitude, f0, delay) in the lowest-index
// element containing it (Newton iteration on the collapsed vertex map) and
// evaluates the basis there.  Points outside every element are an error.
// range (optional, [nsrc][2]) limits the search of source s to elements
// range[2s] <= e < range[2s+1].
int locate_sources(const RefOps& ops, int nsrc, const double* src, const int64_t* range,
                   MeshData& md, std::string& err);

// Locates receiver points xyz [nrec][3] in the K elements whose vertices are
// verts [K][16] (several points may share an element): elem [nrec] and phi
// [nrec][Np] = basis values there.
int locate_receivers(const RefOps& ops, int nrec, const double* xyz, const double* verts,
                     int64_t K, std::vector<int64_t>& elem, std::vector<double>& phi,
                     std::string& err);

// Returns 0 on success or a negative dgpyr_status with a message in err.
// pair_ids (optional, [nverts]) replace the vertex indices when faces are
// paired (periodic meshes give the images of a vertex one id); geometry always
// uses xyz.
int build_mesh(const RefOps& ops, int64_t nverts, const double* xyz, int64_t nelems,
               const int64_t* e2v, const double* rho, const double* kappa, MeshData& md,
               std::string& err, const int64_t* pair_ids = nullptr);

}  // namespace dgpyr
