// Discrete adjoint of the LSRK(5,4) stepping with respect to per-element
// bulk modulus kappa (rho c^2), for a misfit observed at receiver points.
// With dU/dt = F(U, t) = A U + b(t) and the 2N-storage stage
//   R_s = a_s R_{s-1} + dt F(U_{s-1}, t_s),  U_s = U_{s-1} + b_s R_s,
// one step is reversed stage by stage (s = 5 .. 1), given the adjoint Ub of
// the step's final state:
//   Rb += b_s Ub;  grad += dt <Rb, dF/dkappa>;  Ub += dt A^T Rb;  Rb *= a_s,
// with the stage inputs U_{s-1} recomputed from the step's initial state.
// kappa_K enters F as the factor of element K's pressure rows (sources
// included, Section 4.3), giving F_{p,K} / kappa_K, and for alpha > 0 through
// the penalty coefficients of K's faces, {rho c} = (z- + z+)/2 with
// z = sqrt(kappa rho) (k_tau_grad, from the traces of the stage input and of
// M^-1 Kmat Rb).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "context.hpp"
#include "dgpyr.h"
#include "host/mesh.hpp"
#include "host/refops.hpp"
#include "internal.hpp"

using namespace dgpyr::api;

namespace {

template <typename T>
dgpyr_status upload_vec(dgpyr_ctx* c, const std::vector<T>& h, const T** out, const char* what) {
  void* p = nullptr;
  const size_t bytes = h.size() * sizeof(T);
  hipError_t e = hipMalloc(&p, bytes > 0 ? bytes : 16);
  if (e == hipSuccess && bytes) e = hipMemcpy(p, h.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (p) hipFree(p);
    return hip_fail(e, what);
  }
  c->allocs.push_back(p);
  c->device_bytes += (int64_t)bytes;
  *out = static_cast<const T*>(p);
  return DGPYR_OK;
}

}  // namespace

extern "C" {

dgpyr_status dgpyr_set_kappa(dgpyr_ctx* c, const double* kappa) {
  if (dgpyr_status s = check_acoustic(c)) return s;
  if (!kappa) return fail(DGPYR_E_ARG, "kappa is null");
  for (int64_t e = 0; e < c->K; ++e)
    if (!(kappa[e] > 0)) return fail(DGPYR_E_ARG, "kappa must be positive");
  // c_K |dK| / |K| scales with the sound speed c = sqrt(kappa / rho)
  double ilmax = 0.0;
  for (int64_t e = 0; e < c->K; ++e) {
    const double rho = 1.0 / c->mat_host[(size_t)(4 * e + 1)];
    const double kold = c->mat_host[(size_t)(4 * e + 0)];
    c->mat_host[(size_t)(4 * e + 0)] = kappa[e];
    c->mat_host[(size_t)(4 * e + 2)] = std::sqrt(kappa[e] / rho) * rho;
    double& il = c->inv_length[(size_t)e];
    il *= std::sqrt(kappa[e] / kold);
    ilmax = std::max(ilmax, il);
  }
  c->inv_length_max = ilmax;
  hipError_t e = hipMemcpy(const_cast<double*>(c->mesh.mat), c->mat_host.data(),
                           c->mat_host.size() * sizeof(double), hipMemcpyHostToDevice);
  return e == hipSuccess ? DGPYR_OK : hip_fail(e, "upload kappa");
}

dgpyr_status dgpyr_set_receivers(dgpyr_ctx* c, int32_t nrec, const double* xyz) {
  if (dgpyr_status s = check_acoustic(c)) return s;
  if (nrec < 0 || (nrec > 0 && !xyz)) return fail(DGPYR_E_ARG, "bad receiver list");
  if (nrec == 0) {
    c->nrec = 0;
    return DGPYR_OK;
  }
  dgpyr::RefOps ops;
  char msg[256];
  if (!dgpyr::build_refops(c->N, ops, msg, sizeof msg)) return fail(DGPYR_E_STATE, msg);
  std::vector<int64_t> elem;
  std::vector<double> phi;
  std::string err;
  if (int rc = dgpyr::locate_receivers(ops, nrec, xyz, c->verts_host.data(), c->K, elem, phi, err))
    return fail((dgpyr_status)rc, err);
  if (nrec <= c->rec_cap) {  // reuse the reserved or earlier tables
    hipError_t e = hipMemcpy(const_cast<int64_t*>(c->rec_elem), elem.data(),
                             elem.size() * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(const_cast<double*>(c->rec_phi), phi.data(), phi.size() * sizeof(double),
                    hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload receivers");
    c->nrec = nrec;
    return DGPYR_OK;
  }
  if (c->reserved)
    return fail(DGPYR_E_ARG, "more receivers than the reserved DGPYR_MAX_RESERVED_RECEIVERS");
  const int64_t* pe = nullptr;
  const double* pp = nullptr;
  if (dgpyr_status st = upload_vec(c, elem, &pe, "receiver elements")) return st;
  if (dgpyr_status st = upload_vec(c, phi, &pp, "receiver basis values")) return st;
  c->rec_elem = pe;
  c->rec_phi = pp;
  c->nrec = nrec;
  c->rec_cap = nrec;
  return DGPYR_OK;
}

dgpyr_status dgpyr_receivers_sample(dgpyr_ctx* c, const double* U, double* out, void* stream) {
  if (dgpyr_status s = check_acoustic(c)) return s;
  if (!U || (c->nrec > 0 && !out)) return fail(DGPYR_E_ARG, "null array");
  hipError_t e = dgpyr::launch_rec_sample(*c, U, out, (hipStream_t)stream);
  return e == hipSuccess ? DGPYR_OK : hip_fail(e, "receiver sample");
}

dgpyr_status dgpyr_receivers_inject(dgpyr_ctx* c, double* Ubar, const double* coef, void* stream) {
  if (dgpyr_status s = check_acoustic(c)) return s;
  if (!Ubar || (c->nrec > 0 && !coef)) return fail(DGPYR_E_ARG, "null array");
  hipError_t e = dgpyr::launch_rec_inject(*c, Ubar, coef, (hipStream_t)stream);
  return e == hipSuccess ? DGPYR_OK : hip_fail(e, "receiver inject");
}

dgpyr_status dgpyr_adjoint_step(dgpyr_ctx* c, const double* U0, double* Ubar, double* grad,
                                double t0, double dt, void* stream) {
  if (dgpyr_status s = check_acoustic(c)) return s;
  if (!U0 || !Ubar || !grad) return fail(DGPYR_E_ARG, "null array");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = c->K * 4 * c->Np;
  const size_t bytes = (size_t)n * sizeof(double);
  if (!c->adj_work)
    if (dgpyr_status st = alloc(c, 9 * bytes, &c->adj_work, "adjoint step scratch")) return st;
  if (!c->adj_mu)
    if (dgpyr_status st = alloc(c, bytes, &c->adj_mu, "adjoint scratch")) return st;
  if (!c->adj_T)
    if (dgpyr_status st = alloc(c, (size_t)c->K * c->Nfc * 4 * sizeof(double), &c->adj_T,
                                "adjoint trace scratch"))
      return st;
  double* W = c->adj_work;  // W + s n: input of stage s
  double* Rw = W + 5 * n;
  double* Rb = W + 6 * n;
  double* AT = W + 7 * n;
  double* F = W + 8 * n;

  // forward: stage inputs of this step
  hipError_t e = hipMemcpyAsync(W, U0, bytes, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = dgpyr::launch_clock(c->clock, 0.0, false, s);
  c->mesh.clock = c->clock;
  c->mesh.t_base = t0;
  c->mesh.dt_time = dt;
  for (int st = 0; st < 4 && e == hipSuccess; ++st) {
    e = hipMemcpyAsync(W + (st + 1) * n, W + st * n, bytes, hipMemcpyDeviceToDevice, s);
    c->mesh.c_stage = kRkC.c[st];
    if (e == hipSuccess) e = run_stage(c, 1, W + (st + 1) * n, W + (st + 1) * n, Rw, kRkA[st],
                                       kRkB[st], dt, s, nullptr);
  }
  if (e == hipSuccess) e = dgpyr::launch_fill(Rb, n, 0.0, s);
  // reverse
  for (int st = 4; st >= 0 && e == hipSuccess; --st) {
    e = dgpyr::launch_adj_pre(*c, Rb, Ubar, kRkB[st], s);
    // the stage's right-hand side at its input (sources at t0 + c_s dt)
    c->mesh.clock = nullptr;
    c->mesh.t_base = t0 + kRkC.c[st] * dt;
    c->mesh.c_stage = 0.0;
    c->mesh.dt_time = 0.0;
    if (e == hipSuccess) e = run_stage(c, 0, W + st * n, F, nullptr, 0.0, 0.0, 0.0, s, nullptr);
    if (e == hipSuccess) e = dgpyr::launch_kappa_grad(*c, grad, Rb, F, dt, s);
    // the sum-factorised stage keeps (p, u.n) traces: the penalty-coefficient
    // gradient needs all four fields' traces of the stage input
    if (e == hipSuccess && c->sum_factorized)
      e = dgpyr::launch_trace_mfma(*c, W + st * n, c->T, s);
    // A^T Rb
    // (c->T now holds the traces of the stage input W_s)
    if (e == hipSuccess) e = dgpyr::launch_adjoint_scale(*c, Rb, c->adj_mu, s);
    if (e == hipSuccess) e = dgpyr::launch_trace_mfma(*c, c->adj_mu, c->adj_T, s);
    if (e == hipSuccess && c->alpha != 0.0)
      e = dgpyr::launch_tau_grad(*c, grad, c->T, c->adj_T, dt, s);
    if (e == hipSuccess) e = dgpyr::launch_adjoint(*c, c->adj_mu, c->adj_T, AT, s);
    if (e == hipSuccess) e = dgpyr::launch_adj_post(*c, Ubar, Rb, AT, dt, kRkA[st], s);
  }
  return e == hipSuccess ? DGPYR_OK : hip_fail(e, "adjoint step");
}

}  // extern "C"
