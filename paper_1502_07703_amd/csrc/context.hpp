// Library context: reference operators and per-element data on the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "dgpyr.h"
#include "host/mesh.hpp"
#include "host/refops.hpp"

namespace dgpyr {

// Device copies of the reference operators (all FP64, row-major).
struct DevOps {
  const double* DrT;  // [Np][Nc]  d phi_n / dr at volume point q, transposed
  const double* DsT;  // [Np][Nc]
  const double* DtT;  // [Np][Nc]
  const double* V;    // [Nc][Np]  phi_n at volume points
  const double* VfT;  // [Np][Nfc] phi_n at face points, transposed
  const double* Vf;   // [Nfc][Np]
  const double* wv;   // [Nc]      reference volume weights
  const double* wf;   // [Nfc]     face parameter weights
  const double* fa;   // [Nfc]     collapsed a of face points
  const double* fb;   // [Nfc]     collapsed b of face points
  const double* xg;   // [N+1]     Gauss-Legendre nodes
  const double* na;   // [Np]      (a, b) node of each basis function
  const double* nb;   // [Np]
  const double* wwc;  // [Np]      reference mass diagonal w_i^k w_j^k 2/(2k+3)
  const int* perm;    // [10][Nfq] face-point permutations: quad o = 0..7, tri 8..9
};

// Operators in MFMA B-fragment order (see mfma.hpp).  DrF, DsF, DtF, VF and
// LfF are in the precision of the contraction form (double for FP64, float
// for FP32_MFMA); the trace operator VfF is always double.  Consecutive
// fragments are interleaved by lane, KP = 16 / sizeof(element) at a time, so
// that one 16-byte load per lane fetches KP fragments (lane l, slot j):
//   DrF, DsF, DtF  [NTC][NCHP][64][KP]: D[16t + l%16][4(KP cp + j) + l/16]    (derivatives)
//   VF             [NTC][4][NITP][64][KP]: V[16t + 4c + l/16][16(KP up + j) + l%16] (projection)
//   VfF            [NTF][NCHP][64][2]: Vf[16t + l%16][4(2 cp + j) + l/16]     (trace)
//   LfF            [NTF][4][NITP][64][KP]: Vf[16t + 4c + l/16][16(KP up + j) + l%16] (lift)
// with NCHP = ceil(NCH / KP), NITP = ceil(NIT / KP).  Entries outside the
// operator are zero.
struct FragOps {
  const void* DrF;
  const void* DsF;
  const void* DtF;
  const void* VF;
  const void* VfF;
  const void* LfF;
};

// FP64 fragments of the transposed operator (kernels_adjoint.hip), packed as
// FragOps:  VrF [NTC][NCHP][64][2]: V in the derivative layout (interpolation),
// DrP, DsP, DtP [NTC][4][NITP][64][2]: D_rho in the projection layout, LfP the
// lift (V^f) in the projection layout.
struct AdjOps {
  const double* VrF;
  const double* DrP;
  const double* DsP;
  const double* DtP;
  const double* LfP;
};

// Split-BF16 operator fragments (hi and lo parts, bf16 bit patterns), for
// v_mfma_f32_16x16x32_bf16.  Derivative operators, chunk c of 32 basis
// functions, tile t of 16 points:  [t][c][64][8]: D[16t + l%16][32c + 8(l/16) + j];
// projection / lift, chunk t of 32 points, tile u of 16 basis functions:
// [t][u][64][8]: V[32t + 8(l/16) + j][16u + l%16].  Zero outside the operator.
struct Bf16Ops {
  const uint16_t *DrH, *DrL, *DsH, *DsL, *DtH, *DtL;
  const uint16_t *VH, *VL, *LfH, *LfL;
};

// One-dimensional factors for the sum-factorised kernels (host/refops.hpp).
struct SfOps {
  const double* La;  // [k][p][i]
  const double* Da;  // [k][p][i]
  const double* Le;  // [k][2][i]
  const double* G;   // [r][k]
  const double* Gt;  // [r][k]
  const double* Gp;  // [r][k]
  const double* Gb;  // [k]
  const double* Gf;  // [m][k]
  const double* wc;  // [N+1] Gauss-Jacobi(2,0) weights
};

// Per-element device arrays (see host/mesh.hpp for the layouts).
struct DevMesh {
  const double* verts;  // [K][16]
  const int* conn;      // [K][8]
  const double* mat;    // [K][4]: kappa, 1/rho, rho c, time-step scale
  int64_t K;
  int bc;
  double alpha;
  // Point sources (Section 4.3 right-hand side b): src_of[e] is the source
  // index of element e or -1 (NULL: no sources); src_phi [nsrc][Np] =
  // phi_i(xi_s); src_par [nsrc][4] = amplitude, f0, delay, 0.  The stage time
  // of element e is t_base + (clock[0] + c_stage) * dt_time * mat[e][3], with
  // clock the device step counter (NULL reads as 0).
  const int* src_of;
  const double* src_phi;
  const double* src_par;
  const double* clock;
  double t_base;
  double c_stage;
  double dt_time;
};

}  // namespace dgpyr

namespace dgpyr {
// Equation a context discretises.
constexpr int kAcoustic = 0;   // first-order acoustics, 4 fields (Section 4.3)
constexpr int kAdvection = 1;  // linear advection, 1 field (Section 4.1)

// Advection velocity and flux parameter, by value in kernel arguments.
struct AdvParams {
  double beta[3];
  double alpha;
};
}  // namespace dgpyr

struct dgpyr_ctx {
  int N = 0, Np = 0, Nc = 0, Nfq = 0, Nfc = 0;
  int physics = dgpyr::kAcoustic;
  int nfields = 4;                 // fields per element: 4 (acoustics) or 1
  dgpyr::AdvParams adv{};          // advection only
  int64_t K = 0;
  int precision = 0;
  int bc = 0;
  double alpha = 1.0;
  double inv_length_max = 0.0;
  bool hex_groups = false;
  dgpyr::DevOps ops{};
  dgpyr::DevMesh mesh{};
  dgpyr::FragOps frag{};
  dgpyr::AdjOps adj{};
  double* adj_mu = nullptr;  // M^-1 Kmat lam scratch, allocated on first adjoint use
  // reverse-step scratch (allocated on first dgpyr_adjoint_step): stage inputs
  // W[5], forward R, adjoint R, A^T output, stage right-hand side
  double* adj_work = nullptr;
  double* adj_T = nullptr;   // [K][Nfc][4] traces of the adjoint scratch (adjoint step)
  // receivers (dgpyr_set_receivers): element and basis values phi_r [nrec][Np]
  // in device arrays with room for rec_cap points
  int nrec = 0;
  int rec_cap = 0;
  bool reserved = false;  // adjoint and receiver buffers reserved at setup
  const int64_t* rec_elem = nullptr;
  const double* rec_phi = nullptr;
  std::vector<double> verts_host;  // [K][16], for locating receivers
  bool reference_kernels = false;  // plain FP64 VALU kernels instead of MFMA
  bool unfused = false;            // separate matrix-core volume and surface launches
  bool sum_factorized = false;     // FP64 sum-factorised kernels
  bool sf_local = false;           // sum-factorised stage on whole hexahedra (triangle
                                   // traces exchanged in LDS, base traces in T)
  int mfma_groups = 1;             // 4-element groups per wave (fused matrix core)
  bool lds_operators = false;      // stage operator tiles in LDS per workgroup
  int trace_groups = 0;            // 4-element groups per wave of the trace (0: by N)
  dgpyr::SfOps sf{};
  dgpyr::Bf16Ops bf{};
  const double* xc = nullptr;      // [N+1] Gauss-Jacobi(2,0) nodes in c
  double* T = nullptr;    // [K][Nfc][4] face traces
  double* vol = nullptr;  // [K][4][Np] volume contribution
  double* clock = nullptr;  // device step counter (source times)
  unsigned long long* watch = nullptr;  // NaN/Inf watchdog: first bad step, or all
                                        // ones; null without DGPYR_FLAG_WATCHDOG
  int64_t watch_steps = 0;              // steps checked since the last query
  int nsrc = 0;
  int64_t device_bytes = 0;
  int device = 0;  // HIP device the context was set up on
  std::vector<void*> allocs;
  // host copies kept for batches (per-problem time steps): c_K |dK| / |K| and
  // the material rows [K][4] whose last entry scales the time step
  std::vector<double> inv_length;
  std::vector<double> mat_host;
};

namespace dgpyr {

// Kernel launchers (kernels_fp64.hip).  mode 0: out = dU/dt; mode 1: LSRK
// stage R <- ra R + dt rhs (R not read when ra == 0), out(U) <- out + rb R.
hipError_t launch_trace(const dgpyr_ctx& c, const double* U, double* T, hipStream_t s);
hipError_t launch_volume(const dgpyr_ctx& c, const double* U, double* vol, hipStream_t s);
hipError_t launch_surface(const dgpyr_ctx& c, int mode, const double* T, const double* vol,
                          double* out, double* R, double ra, double rb, double dt, hipStream_t s);
// Initial data and evaluation (kernels_aux.hip).
hipError_t launch_points(const dgpyr_ctx& c, double* xyz, double* wJ, hipStream_t s);
hipError_t launch_clock(double* clock, double value, bool add, hipStream_t s);
hipError_t launch_fill(double* x, int64_t n, double value, hipStream_t s);
hipError_t launch_nonfinite(const double* x, int64_t n, unsigned long long step,
                            unsigned long long* first_bad, hipStream_t s);
// Transposed operator (kernels_adjoint.hip).
hipError_t launch_adjoint_scale(const dgpyr_ctx& c, const double* lam, double* mu, hipStream_t s);
hipError_t launch_adjoint(const dgpyr_ctx& c, const double* mu, const double* T, double* out,
                          hipStream_t s);
hipError_t launch_rec_sample(const dgpyr_ctx& c, const double* U, double* out, hipStream_t s);
hipError_t launch_rec_inject(const dgpyr_ctx& c, double* Ub, const double* coef, hipStream_t s);
hipError_t launch_adj_pre(const dgpyr_ctx& c, double* Rb, const double* Ub, double bs,
                          hipStream_t s);
hipError_t launch_adj_post(const dgpyr_ctx& c, double* Ub, double* Rb, const double* ATRb,
                           double dt, double as, hipStream_t s);
hipError_t launch_kappa_grad(const dgpyr_ctx& c, double* grad, const double* Rb, const double* F,
                             double dt, hipStream_t s);
// kappa derivative through the penalty coefficients: traces of the forward
// state TW and of M^-1 Kmat Rb TM ([K][Nfc][4] each).
hipError_t launch_tau_grad(const dgpyr_ctx& c, double* grad, const double* TW, const double* TM,
                           double dt, hipStream_t s);
hipError_t launch_project(const dgpyr_ctx& c, const double* f, double* U, hipStream_t s);
hipError_t launch_eval(const dgpyr_ctx& c, const double* U, double* f, hipStream_t s);
// Matrix-core kernels (kernels_mfma.hip).
hipError_t launch_volume_mfma(const dgpyr_ctx& c, const double* U, double* vol, hipStream_t s);
hipError_t launch_trace_mfma(const dgpyr_ctx& c, const double* U, double* T, hipStream_t s);
// Sum-factorised FP64 kernels (kernels_sumfact.hip).  On whole hexahedra
// (sf_local) the traces are (p, u.n) pairs of the base faces, [K][(N+1)^2][2];
// otherwise of all five faces, [K][Nfc][2].
hipError_t launch_sf_trace(const dgpyr_ctx& c, const double* U, double* T2, hipStream_t s);
hipError_t launch_sf_stage(const dgpyr_ctx& c, int mode, const double* U, const double* T2,
                           double* out, double* R, double ra, double rb, double dt, hipStream_t s);
// Whether whole hexahedra fit one workgroup at the context's N.
bool sf_local_possible(const dgpyr_ctx& c);
// LDS, private memory and block size of the sum-factorised kernels against the
// device's limits; E_UNSUPPORTED with a message when a kernel does not fit.
dgpyr_status sf_check_resources(const dgpyr_ctx& c, std::string& msg);
// Split-BF16 fused stage (kernels_bf16.hip).
hipError_t launch_stage_bf16(const dgpyr_ctx& c, int mode, const double* U, const double* T,
                             double* out, double* R, double ra, double rb, double dt,
                             hipStream_t s);
// Advection (kernels_advection.hip): traces [K][Nfc] and the fused stage.
hipError_t launch_adv_trace(const dgpyr_ctx& c, const double* U, double* T, hipStream_t s);
hipError_t launch_adv_stage(const dgpyr_ctx& c, int mode, const double* U, const double* T,
                            double* out, double* R, double ra, double rb, double dt,
                            hipStream_t s);
// Fused volume + surface + inverse mass (+ RK stage) in one launch.
hipError_t launch_stage_mfma(const dgpyr_ctx& c, int mode, const double* U, const double* T,
                             double* out, double* R, double ra, double rb, double dt,
                             hipStream_t s);
hipError_t launch_surface_mfma(const dgpyr_ctx& c, int mode, const double* T, const double* vol,
                               double* out, double* R, double ra, double rb, double dt,
                               hipStream_t s);

}  // namespace dgpyr
