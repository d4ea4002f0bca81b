// CPU run of the library's sum-factorised kernels (kernels_sumfact.hip,
// included unchanged and compiled for the host against the stand-in
// hip/hip_runtime.h of this folder), for checking their indexing and results
// under AddressSanitizer.  Test infrastructure, not part of the library.
//
//   emu_sumfact <input> <output>
// input (little-endian): int64 N, nverts, nelems, bc, nsteps; double alpha, dt;
//   xyz [nverts][3], int64 e2v [nelems][5], rho [nelems], kappa [nelems],
//   U [nelems][4][Np].
// nsteps = 0: output is the right-hand side [nelems][4][Np]; nsteps > 0: the
// state after nsteps LSRK(5,4) steps of size dt.  The first output int64 is
// 1 if the whole-hexahedron (LDS-exchange) variant ran, else 0.
#include "kernels_sumfact.hip"

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host/mesh.hpp"
#include "host/refops.hpp"

namespace {

template <typename T>
bool rd(FILE* f, T* p, size_t n) {
  return std::fread(p, sizeof(T), n, f) == n;
}

// Carpenter-Kennedy RK(5,4) 2N-storage coefficients (published values).
const double kA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                      -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double kB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                      1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                      2277821191437.0 / 14882151754819.0};

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: emu_sumfact <input> <output>\n");
    return 2;
  }
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t hdr[5];
  double par[2];
  if (!rd(f, hdr, 5) || !rd(f, par, 2)) return 2;
  const int N = (int)hdr[0];
  const int64_t nverts = hdr[1], K = hdr[2];
  const int bc = (int)hdr[3], nsteps = (int)hdr[4];
  const int Np = dgpyr::n_basis(N);
  std::vector<double> xyz((size_t)nverts * 3), rho((size_t)K), kap((size_t)K);
  std::vector<int64_t> e2v((size_t)K * 5);
  std::vector<double> U((size_t)K * 4 * Np);
  if (!rd(f, xyz.data(), xyz.size()) || !rd(f, e2v.data(), e2v.size()) ||
      !rd(f, rho.data(), rho.size()) || !rd(f, kap.data(), kap.size()) ||
      !rd(f, U.data(), U.size()))
    return 2;
  std::fclose(f);

  dgpyr::RefOps ops;
  char msg[256];
  if (!dgpyr::build_refops(N, ops, msg, sizeof msg)) {
    std::fprintf(stderr, "%s\n", msg);
    return 3;
  }
  dgpyr::MeshData md;
  std::string err;
  if (dgpyr::build_mesh(ops, nverts, xyz.data(), K, e2v.data(), rho.data(), kap.data(), md,
                        err) != 0) {
    std::fprintf(stderr, "%s\n", err.c_str());
    return 3;
  }
  std::vector<int> perm((size_t)10 * ops.Nfq);
  for (int o = 0; o < 8; ++o) dgpyr::quad_perm(N, o, &perm[(size_t)o * ops.Nfq]);
  for (int o = 0; o < 2; ++o) dgpyr::tri_perm(N, o, &perm[(size_t)(8 + o) * ops.Nfq]);

  dgpyr_ctx c;
  c.N = N;
  c.Np = Np;
  c.Nc = ops.Nc;
  c.Nfq = ops.Nfq;
  c.Nfc = ops.Nfc;
  c.K = K;
  c.bc = bc;
  c.alpha = par[0];
  c.sum_factorized = true;
  c.ops.wf = ops.wf.data();
  c.ops.fa = ops.fa.data();
  c.ops.fb = ops.fb.data();
  c.ops.xg = ops.xg.data();
  c.ops.na = ops.na.data();
  c.ops.nb = ops.nb.data();
  c.ops.wwc = ops.wwc.data();
  c.ops.perm = perm.data();
  c.sf = dgpyr::SfOps{ops.sfLa.data(), ops.sfDa.data(), ops.sfLe.data(), ops.sfG.data(),
                      ops.sfGt.data(), ops.sfGp.data(), ops.sfGb.data(), ops.sfGf.data(),
                      ops.wc.data()};
  c.mesh.verts = md.verts.data();
  c.mesh.conn = md.conn.data();
  c.mesh.mat = md.mat.data();
  c.mesh.K = K;
  c.mesh.bc = bc;
  c.mesh.alpha = par[0];
  c.sf_local = md.hex_groups && dgpyr::sf_local_possible(c);
  std::string rmsg;
  if (dgpyr::sf_check_resources(c, rmsg) != DGPYR_OK) {
    std::fprintf(stderr, "%s\n", rmsg.c_str());
    return 3;
  }

  // exactly sized buffers (AddressSanitizer flags any access past them)
  std::vector<double> T2(c.sf_local ? (size_t)K * ops.Nfq * 2 : (size_t)K * ops.Nfc * 2);
  std::vector<double> out((size_t)K * 4 * Np), R(nsteps > 0 ? (size_t)K * 4 * Np : 0);
  if (nsteps == 0) {
    if (dgpyr::launch_sf_trace(c, U.data(), T2.data(), nullptr) != hipSuccess) return 4;
    if (dgpyr::launch_sf_stage(c, 0, U.data(), T2.data(), out.data(), nullptr, 0.0, 0.0, 0.0,
                               nullptr) != hipSuccess)
      return 4;
  } else {
    for (int n = 0; n < nsteps; ++n)
      for (int s = 0; s < 5; ++s) {
        if (dgpyr::launch_sf_trace(c, U.data(), T2.data(), nullptr) != hipSuccess) return 4;
        if (dgpyr::launch_sf_stage(c, 1, U.data(), T2.data(), U.data(), R.data(), kA[s], kB[s],
                                   par[1], nullptr) != hipSuccess)
          return 4;
      }
    out = U;
  }
  FILE* g = std::fopen(argv[2], "wb");
  if (!g) return 2;
  const int64_t local = c.sf_local ? 1 : 0;
  std::fwrite(&local, sizeof local, 1, g);
  std::fwrite(out.data(), sizeof(double), out.size(), g);
  std::fclose(g);
  return 0;
}
