// Setup of linear-advection contexts (Section 4.1): same reference data and
// geometry as the acoustic path, faces paired through caller-given vertex
// identities (periodic meshes), one field per element.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>

#include "context.hpp"
#include "dgpyr.h"
#include "host/mesh.hpp"
#include "host/refops.hpp"
#include "internal.hpp"

using namespace dgpyr::api;

namespace {

// Host part shared by the setup and the host-only builder: argument checks
// on the mesh, reference data, geometry and face pairing.
dgpyr_status adv_host_build(const dgpyr_advection_mesh* mesh, int32_t N, dgpyr::RefOps& ops,
                            dgpyr::MeshData& md) {
  if (!mesh) return fail(DGPYR_E_ARG, "mesh is null");
  if (!mesh->xyz || !mesh->e2v || mesh->nverts <= 0 || mesh->nelems <= 0)
    return fail(DGPYR_E_ARG, "mesh arrays must be non-null with positive sizes");
  if (mesh->nelems > (int64_t)0x7fffffff) return fail(DGPYR_E_ARG, "more than 2^31-1 elements");
  if (N < 0 || N > DGPYR_MAX_ORDER) return fail(DGPYR_E_ORDER, "N must be in [0, 8]");
  char msg[256];
  if (!dgpyr::build_refops(N, ops, msg, sizeof msg)) return fail(DGPYR_E_STATE, msg);
  std::string err;
  int rc = dgpyr::build_mesh(ops, mesh->nverts, mesh->xyz, mesh->nelems, mesh->e2v, nullptr,
                             nullptr, md, err, mesh->pair_ids);
  if (rc != 0) return fail((dgpyr_status)rc, err);
  return DGPYR_OK;
}

}  // namespace

extern "C" {

dgpyr_status dgpyr_host_advection_mesh(const dgpyr_advection_mesh* mesh, int32_t N, int32_t* nbr,
                                       int32_t* nface) {
  dgpyr::RefOps ops;
  dgpyr::MeshData md;
  if (dgpyr_status st = adv_host_build(mesh, N, ops, md)) return st;
  for (int64_t e = 0; e < md.K; ++e)
    for (int f = 0; f < 5; ++f) {
      const int32_t nb = md.conn[(size_t)e * 8 + f];
      if (nbr) nbr[5 * e + f] = nb;
      if (nface)
        nface[5 * e + f] = nb < 0 ? -1 : (int32_t)(((uint32_t)md.conn[(size_t)e * 8 + 5] >> (6 * f)) & 7u);
    }
  return DGPYR_OK;
}

dgpyr_status dgpyr_advection_setup(const dgpyr_advection_mesh* mesh, int32_t N,
                                   const dgpyr_advection_opts* opts, void* stream,
                                   dgpyr_ctx** out) {
  (void)stream;
  if (!out) return fail(DGPYR_E_ARG, "out is null");
  *out = nullptr;
  if (!mesh || !opts) return fail(DGPYR_E_ARG, "mesh or opts is null");
  if (opts->flags != 0) return fail(DGPYR_E_ARG, "unknown flag bits");
  if (!(opts->alpha >= 0.0 && opts->alpha <= 1.0)) return fail(DGPYR_E_ARG, "alpha must be in [0, 1]");
  double bb = 0.0;
  for (int d = 0; d < 3; ++d) {
    if (!std::isfinite(opts->beta[d])) return fail(DGPYR_E_ARG, "beta must be finite");
    bb += opts->beta[d] * opts->beta[d];
  }
  if (!(bb > 0.0)) return fail(DGPYR_E_ARG, "beta must be non-zero");
  if (opts->precision != DGPYR_FP64)
    return fail(DGPYR_E_UNSUPPORTED, "advection is built in FP64 only");

  dgpyr::RefOps ops;
  dgpyr::MeshData md;
  if (dgpyr_status st = adv_host_build(mesh, N, ops, md)) return st;
  dgpyr_ctx* c = new (std::nothrow) dgpyr_ctx();
  if (!c) return fail(DGPYR_E_OOM, "host allocation failed");
  const double bnorm = std::sqrt(bb);
  c->physics = dgpyr::kAdvection;
  c->nfields = 1;
  for (int d = 0; d < 3; ++d) c->adv.beta[d] = opts->beta[d];
  c->adv.alpha = opts->alpha;
  c->N = N;
  c->Np = ops.Np;
  c->Nc = ops.Nc;
  c->Nfq = ops.Nfq;
  c->Nfc = ops.Nfc;
  c->K = mesh->nelems;
  c->precision = DGPYR_FP64;
  c->bc = DGPYR_BC_WALL;
  c->alpha = opts->alpha;
  // |dK| / |K| scaled by the speed |beta| (c = 1 in the mesh builder)
  c->inv_length = md.inv_length;
  for (double& v : c->inv_length) v *= bnorm;
  c->inv_length_max = md.inv_length_max * bnorm;
  c->hex_groups = md.hex_groups;
  c->mat_host = md.mat;
  c->verts_host = md.verts;
  dgpyr_status st = upload_context(c, ops, md);
  if (st != DGPYR_OK) {
    free_ctx(c);
    return st;
  }
  c->mesh.K = c->K;
  c->mesh.bc = c->bc;
  c->mesh.alpha = c->alpha;
  *out = c;
  return DGPYR_OK;
}

}  // extern "C"
