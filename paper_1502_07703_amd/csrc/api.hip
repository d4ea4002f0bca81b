// C ABI of the library: setup (host FP64 builders + upload), state layout,
// right-hand side and LSRK stepping.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "context.hpp"
#include "dgpyr.h"
#include "host/mesh.hpp"
#include "host/refops.hpp"
#include "internal.hpp"

// Scratch of dgpyr_adjoint_rhs_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code never passes the name
// `scratch` to a kernel or copy (on the host it is only a stand-in for the
// symbol); it uses the per-device address that set-up obtains from
// hipGetSymbolAddress with that device current.
constexpr size_t kScratchDoubles = DGPYR_NOALLOC_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace dgpyr {
namespace api {

thread_local std::string g_err;

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` per device
}  // namespace

// Looks up the address of `scratch` on the current device (once per device).
dgpyr_status scratch_for_current_device(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(DGPYR_E_UNSUPPORTED, "device index too large");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return DGPYR_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  if (!p) return fail(DGPYR_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
  g_scratch_ptr[dev] = static_cast<double*>(p);
  return DGPYR_OK;
}

double* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}

dgpyr_status fail(dgpyr_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

dgpyr_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? DGPYR_E_OOM : DGPYR_E_HIP;
}

// Carpenter-Kennedy 2N-storage RK(5,4) coefficients.
extern const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
extern const double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

StageTimes::StageTimes() {
  double u = 0.0, r = 0.0;
  for (int s = 0; s < 5; ++s) {
    c[s] = u;
    r = kRkA[s] * r + 1.0;
    u += kRkB[s] * r;
  }
}
extern const StageTimes kRkC;
const StageTimes kRkC;

template <typename T>
dgpyr_status upload(dgpyr_ctx* c, const std::vector<T>& h, const T** out, const char* what) {
  void* p = nullptr;
  const size_t bytes = h.size() * sizeof(T);
  hipError_t e = hipMalloc(&p, bytes > 0 ? bytes : 16);
  if (e != hipSuccess) return hip_fail(e, what);
  c->allocs.push_back(p);
  c->device_bytes += (int64_t)bytes;
  if (bytes) {
    e = hipMemcpy(p, h.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, what);
  }
  *out = static_cast<const T*>(p);
  return DGPYR_OK;
}

dgpyr_status alloc(dgpyr_ctx* c, size_t bytes, double** out, const char* what) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes > 0 ? bytes : 16);
  if (e != hipSuccess) return hip_fail(e, what);
  c->allocs.push_back(p);
  c->device_bytes += (int64_t)bytes;
  *out = static_cast<double*>(p);
  return DGPYR_OK;
}

std::vector<double> transpose(const std::vector<double>& A, int rows, int cols) {
  std::vector<double> B((size_t)rows * cols);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) B[(size_t)c * rows + r] = A[(size_t)r * cols + c];
  return B;
}

// Times launches with a ring of HIP event pairs; the host only waits on an
// event pair when it is about to reuse it, so it stays far ahead of the GPU.
struct LaunchTimer {
  static constexpr int kRing = 256;
  hipStream_t s;
  int nk;
  double* ms;
  int64_t* count;
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;
  int64_t n = 0;
  hipError_t err = hipSuccess;
  LaunchTimer(hipStream_t s_, int nk_, double* ms_, int64_t* cnt_) : s(s_), nk(nk_), ms(ms_), count(cnt_) {
    ev.resize(2 * kRing, nullptr);
    kind.assign(kRing, -1);
    for (auto& e : ev)
      if (err == hipSuccess) err = hipEventCreate(&e);
  }
  ~LaunchTimer() {
    for (auto& e : ev)
      if (e) hipEventDestroy(e);
  }
  void retire(int slot) {
    if (kind[slot] < 0) return;
    float t = 0.f;
    hipError_t e = hipEventSynchronize(ev[2 * slot + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[2 * slot], ev[2 * slot + 1]);
    if (e != hipSuccess && err == hipSuccess) err = e;
    if (kind[slot] < nk) {
      ms[kind[slot]] += t;
      count[kind[slot]] += 1;
    }
    kind[slot] = -1;
  }
  void begin(int k) {
    const int slot = (int)(n % kRing);
    retire(slot);
    kind[slot] = k;
    hipError_t e = hipEventRecord(ev[2 * slot], s);
    if (e != hipSuccess && err == hipSuccess) err = e;
  }
  void end() {
    const int slot = (int)(n % kRing);
    hipError_t e = hipEventRecord(ev[2 * slot + 1], s);
    if (e != hipSuccess && err == hipSuccess) err = e;
    ++n;
  }
  void drain() {
    for (int i = 0; i < kRing; ++i) retire(i);
  }
};

// Default 4-element groups per wave of the fused stage kernel.  Measured at
// 384000 pyramids, N = 4: one group compiled for three waves per SIMD takes
// 3.09 ms (FP64) and 2.47 ms (FP32) against 3.37 ms and 2.89 ms for two
// groups at two waves per SIMD.
int default_groups(int N, int precision) {
  (void)N;
  (void)precision;
  return 1;
}

// Kernel kinds per path, in dgpyr_step_timed order.
const char* kNamesFused = "trace;stage";
const char* kNamesSplit = "trace;volume;surface_update";

const char* kernel_names(const dgpyr_ctx* c) {
  if (c->physics == dgpyr::kAdvection) return kNamesFused;
  return (c->reference_kernels || c->unfused) ? kNamesSplit : kNamesFused;
}

// One LSRK stage (mode 1) or one right-hand side evaluation (mode 0).
// Default path: matrix-core trace, then the fused stage kernel.  Split paths
// (reference vector-ALU kernels, or the unfused matrix-core kernels): trace,
// volume, surface + update.
hipError_t run_stage(dgpyr_ctx* c, int mode, const double* U, double* out, double* R, double ra,
                     double rb, double dt, hipStream_t s, LaunchTimer* tm) {
  if (c->physics == dgpyr::kAdvection) {
    if (tm) tm->begin(0);
    hipError_t e = dgpyr::launch_adv_trace(*c, U, c->T, s);
    if (tm) tm->end();
    if (e != hipSuccess) return e;
    if (tm) tm->begin(1);
    e = dgpyr::launch_adv_stage(*c, mode, U, c->T, out, R, ra, rb, dt, s);
    if (tm) tm->end();
    return e;
  }
  if (c->sum_factorized) {
    // traces as (p, u.n) pairs: base faces only on whole hexahedra
    if (tm) tm->begin(0);
    hipError_t e = dgpyr::launch_sf_trace(*c, U, c->T, s);
    if (tm) tm->end();
    if (e != hipSuccess) return e;
    if (tm) tm->begin(1);
    e = dgpyr::launch_sf_stage(*c, mode, U, c->T, out, R, ra, rb, dt, s);
    if (tm) tm->end();
    return e;
  }
  if (tm) tm->begin(0);
  hipError_t e = c->reference_kernels ? dgpyr::launch_trace(*c, U, c->T, s)
                                      : dgpyr::launch_trace_mfma(*c, U, c->T, s);
  if (tm) tm->end();
  if (e != hipSuccess) return e;
  if (!c->reference_kernels && !c->unfused) {
    if (tm) tm->begin(1);
    e = c->precision == DGPYR_SPLIT_BF16
            ? dgpyr::launch_stage_bf16(*c, mode, U, c->T, out, R, ra, rb, dt, s)
            : dgpyr::launch_stage_mfma(*c, mode, U, c->T, out, R, ra, rb, dt, s);
    if (tm) tm->end();
    return e;
  }
  if (tm) tm->begin(1);
  e = c->reference_kernels ? dgpyr::launch_volume(*c, U, c->vol, s)
                           : dgpyr::launch_volume_mfma(*c, U, c->vol, s);
  if (tm) tm->end();
  if (e != hipSuccess) return e;
  if (tm) tm->begin(2);
  e = c->reference_kernels
          ? dgpyr::launch_surface(*c, mode, c->T, c->vol, out, R, ra, rb, dt, s)
          : dgpyr::launch_surface_mfma(*c, mode, c->T, c->vol, out, R, ra, rb, dt, s);
  if (tm) tm->end();
  return e;
}

// Operator fragments in MFMA B order, packed so that each lane reads KP =
// 16 / sizeof(T) consecutive fragments with one 16-byte load (layouts in
// context.hpp).  Entries outside the operator (and padding) are zero.
template <typename T>
constexpr int pack_of() { return (int)(16 / sizeof(T)); }

template <typename T>
std::vector<T> frag_rows(const std::vector<double>& Op, int P, int Np) {
  // B_c[k][j] = Op[16t + j][4c + k], tiles t over P points, chunks c over Np;
  // stored [t][c / KP][lane][c % KP]
  constexpr int KP = pack_of<T>();
  const int NT = (P + 15) / 16, NCH = (Np + 3) / 4, NCHP = (NCH + KP - 1) / KP;
  std::vector<T> out((size_t)NT * NCHP * 64 * KP, (T)0);
  for (int t = 0; t < NT; ++t)
    for (int c = 0; c < NCH; ++c)
      for (int l = 0; l < 64; ++l) {
        const int q = 16 * t + l % 16, n = 4 * c + l / 16;
        if (q < P && n < Np)
          out[(((size_t)t * NCHP + c / KP) * 64 + l) * KP + c % KP] = (T)Op[(size_t)q * Np + n];
      }
  return out;
}

template <typename T>
std::vector<T> frag_proj(const std::vector<double>& Op, int P, int Np) {
  // B_u[k][j] = Op[16t + 4c + k][16u + j], tiles t over P points, c = 0..3,
  // u over Np; stored [t][c][u / KP][lane][u % KP]
  constexpr int KP = pack_of<T>();
  const int NT = (P + 15) / 16, NIT = (Np + 15) / 16, NITP = (NIT + KP - 1) / KP;
  std::vector<T> out((size_t)NT * 4 * NITP * 64 * KP, (T)0);
  for (int t = 0; t < NT; ++t)
    for (int c = 0; c < 4; ++c)
      for (int u = 0; u < NIT; ++u)
        for (int l = 0; l < 64; ++l) {
          const int q = 16 * t + 4 * c + l / 16, i = 16 * u + l % 16;
          if (q < P && i < Np)
            out[((((size_t)t * 4 + c) * NITP + u / KP) * 64 + l) * KP + u % KP] =
                (T)Op[(size_t)q * Np + i];
        }
  return out;
}

template <typename T>
dgpyr_status upload_frags(dgpyr_ctx* c, const dgpyr::RefOps& o) {
  dgpyr_status st = DGPYR_OK;
  const T* p = nullptr;
  if (st == DGPYR_OK && (st = upload(c, frag_rows<T>(o.Dr, o.Nc, o.Np), &p, "DrF")) == DGPYR_OK) c->frag.DrF = p;
  if (st == DGPYR_OK && (st = upload(c, frag_rows<T>(o.Ds, o.Nc, o.Np), &p, "DsF")) == DGPYR_OK) c->frag.DsF = p;
  if (st == DGPYR_OK && (st = upload(c, frag_rows<T>(o.Dt, o.Nc, o.Np), &p, "DtF")) == DGPYR_OK) c->frag.DtF = p;
  if (st == DGPYR_OK && (st = upload(c, frag_proj<T>(o.V, o.Nc, o.Np), &p, "VF")) == DGPYR_OK) c->frag.VF = p;
  const double* pd = nullptr;
  if (st == DGPYR_OK && (st = upload(c, frag_rows<double>(o.Vf, o.Nfc, o.Np), &pd, "VfF")) == DGPYR_OK)
    c->frag.VfF = pd;
  if (st == DGPYR_OK && (st = upload(c, frag_proj<T>(o.Vf, o.Nfc, o.Np), &p, "LfF")) == DGPYR_OK) c->frag.LfF = p;
  return st;
}

// bf16 bit pattern of a float, round to nearest even (finite inputs).
uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Split-BF16 fragments (layouts in context.hpp): hi = bf16(x), lo = bf16(x - hi).
void frag_bf16_rows(const std::vector<double>& Op, int P, int Np, std::vector<uint16_t>& hi,
                    std::vector<uint16_t>& lo) {
  const int NT = (P + 15) / 16, NC = (Np + 31) / 32;
  hi.assign((size_t)NT * NC * 64 * 8, 0);
  lo.assign(hi.size(), 0);
  for (int t = 0; t < NT; ++t)
    for (int c = 0; c < NC; ++c)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 8; ++j) {
          const int q = 16 * t + l % 16, n = 32 * c + 8 * (l / 16) + j;
          if (q >= P || n >= Np) continue;
          const double x = Op[(size_t)q * Np + n];
          const size_t idx = (((size_t)t * NC + c) * 64 + l) * 8 + j;
          hi[idx] = bf16_bits((float)x);
          lo[idx] = bf16_bits((float)(x - (double)bf16_value(hi[idx])));
        }
}

void frag_bf16_proj(const std::vector<double>& Op, int P, int Np, std::vector<uint16_t>& hi,
                    std::vector<uint16_t>& lo) {
  const int NT = (P + 31) / 32, NIT = (Np + 15) / 16;
  hi.assign((size_t)NT * NIT * 64 * 8, 0);
  lo.assign(hi.size(), 0);
  for (int t = 0; t < NT; ++t)
    for (int u = 0; u < NIT; ++u)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 8; ++j) {
          const int q = 32 * t + 8 * (l / 16) + j, i = 16 * u + l % 16;
          if (q >= P || i >= Np) continue;
          const double x = Op[(size_t)q * Np + i];
          const size_t idx = (((size_t)t * NIT + u) * 64 + l) * 8 + j;
          hi[idx] = bf16_bits((float)x);
          lo[idx] = bf16_bits((float)(x - (double)bf16_value(hi[idx])));
        }
}

dgpyr_status upload_bf16(dgpyr_ctx* c, const dgpyr::RefOps& o) {
  dgpyr_status st = DGPYR_OK;
  std::vector<uint16_t> h, l;
  const double* pd = nullptr;
  if (st == DGPYR_OK && (st = upload(c, frag_rows<double>(o.Vf, o.Nfc, o.Np), &pd, "VfF")) == DGPYR_OK)
    c->frag.VfF = pd;
  struct Item { const std::vector<double>* op; int P; bool rows; const uint16_t** H; const uint16_t** L; };
  const Item items[] = {{&o.Dr, o.Nc, true, &c->bf.DrH, &c->bf.DrL},
                        {&o.Ds, o.Nc, true, &c->bf.DsH, &c->bf.DsL},
                        {&o.Dt, o.Nc, true, &c->bf.DtH, &c->bf.DtL},
                        {&o.V, o.Nc, false, &c->bf.VH, &c->bf.VL},
                        {&o.Vf, o.Nfc, false, &c->bf.LfH, &c->bf.LfL}};
  for (const Item& it : items) {
    if (st != DGPYR_OK) break;
    if (it.rows) frag_bf16_rows(*it.op, it.P, o.Np, h, l);
    else frag_bf16_proj(*it.op, it.P, o.Np, h, l);
    st = upload(c, h, it.H, "bf16 hi");
    if (st == DGPYR_OK) st = upload(c, l, it.L, "bf16 lo");
  }
  return st;
}

void free_ctx(dgpyr_ctx* c) {
  if (!c) return;
  for (void* p : c->allocs) hipFree(p);
  delete c;
}

dgpyr_status check_ctx(const dgpyr_ctx* c) {
  if (!c) return fail(DGPYR_E_ARG, "null context");
  return DGPYR_OK;
}

dgpyr_status check_acoustic(const dgpyr_ctx* c) {
  if (dgpyr_status s = check_ctx(c)) return s;
  if (c->physics != dgpyr::kAcoustic)
    return fail(DGPYR_E_UNSUPPORTED, "this call is built for the acoustic equations only");
  return DGPYR_OK;
}

}  // namespace api
}  // namespace dgpyr

using namespace dgpyr::api;

extern "C" {

const char* dgpyr_status_string(dgpyr_status s) {
  switch (s) {
    case DGPYR_OK: return "ok";
    case DGPYR_E_ARG: return "invalid argument";
    case DGPYR_E_ORDER: return "polynomial degree out of range";
    case DGPYR_E_MESH: return "invalid mesh geometry";
    case DGPYR_E_NONCONFORMING: return "non-conforming mesh";
    case DGPYR_E_HIP: return "HIP runtime error";
    case DGPYR_E_OOM: return "out of device memory";
    case DGPYR_E_STATE: return "invalid context state";
    case DGPYR_E_UNSUPPORTED: return "unsupported option";
  }
  return "unknown status";
}

const char* dgpyr_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace dgpyr {
namespace api {

// Setup shared by dgpyr_setup and the batch: dtscale (optional, [K]) is the
// per-element time-step scale; src_range (optional) limits each source's
// element search.
// Per-element geometry, connectivity, materials, sources and the step clock.
dgpyr_status upload_mesh(dgpyr_ctx* c, const dgpyr::MeshData& md) {
  dgpyr_status st = DGPYR_OK;
  if (st == DGPYR_OK) st = upload(c, md.verts, &c->mesh.verts, "verts");
  if (st == DGPYR_OK) st = upload(c, md.conn, &c->mesh.conn, "conn");
  if (st == DGPYR_OK) st = upload(c, md.mat, &c->mesh.mat, "mat");
  if (st == DGPYR_OK && md.nsrc > 0) {
    c->nsrc = md.nsrc;
    st = upload(c, md.src_of, &c->mesh.src_of, "src_of");
    if (st == DGPYR_OK) st = upload(c, md.src_phi, &c->mesh.src_phi, "src_phi");
    if (st == DGPYR_OK) st = upload(c, md.src_par, &c->mesh.src_par, "src_par");
  }
  if (st == DGPYR_OK) {
    std::vector<double> zero(2, 0.0);
    const double* pc = nullptr;
    st = upload(c, zero, &pc, "clock");
    c->clock = const_cast<double*>(pc);
  }
  return st;
}

// Reference operators, fragments, per-element data and work buffers of a
// context whose sizes, physics and precision are set.
dgpyr_status upload_context(dgpyr_ctx* c, const dgpyr::RefOps& ops, const dgpyr::MeshData& md) {
  std::vector<int> perm((size_t)10 * ops.Nfq);
  for (int o = 0; o < 8; ++o) dgpyr::quad_perm(c->N, o, &perm[(size_t)o * ops.Nfq]);
  for (int o = 0; o < 2; ++o) dgpyr::tri_perm(c->N, o, &perm[(size_t)(8 + o) * ops.Nfq]);

  dgpyr_status st = DGPYR_OK;
#define UP(vec, field) \
  if (st == DGPYR_OK) st = upload(c, vec, &c->ops.field, #field);
  UP(transpose(ops.Dr, ops.Nc, ops.Np), DrT)
  UP(transpose(ops.Ds, ops.Nc, ops.Np), DsT)
  UP(transpose(ops.Dt, ops.Nc, ops.Np), DtT)
  UP(ops.V, V)
  UP(transpose(ops.Vf, ops.Nfc, ops.Np), VfT)
  UP(ops.Vf, Vf)
  UP(ops.wv, wv)
  UP(ops.wf, wf)
  UP(ops.fa, fa)
  UP(ops.fb, fb)
  UP(ops.xg, xg)
  UP(ops.na, na)
  UP(ops.nb, nb)
  UP(ops.wwc, wwc)
  UP(perm, perm)
#undef UP
  if (st == DGPYR_OK) st = upload(c, ops.xc, &c->xc, "xc");
  if (st != DGPYR_OK || c->physics != dgpyr::kAcoustic) {
    // advection: FP64 fragments only
    if (st == DGPYR_OK) st = upload_frags<double>(c, ops);
    if (st == DGPYR_OK) st = upload_mesh(c, md);
    if (st == DGPYR_OK)
      st = alloc(c, (size_t)c->K * c->Nfc * c->nfields * sizeof(double), &c->T, "trace buffer");
    return st;
  }
  if (st == DGPYR_OK) st = upload(c, ops.sfLa, &c->sf.La, "sfLa");
  if (st == DGPYR_OK) st = upload(c, ops.sfDa, &c->sf.Da, "sfDa");
  if (st == DGPYR_OK) st = upload(c, ops.sfLe, &c->sf.Le, "sfLe");
  if (st == DGPYR_OK) st = upload(c, ops.sfG, &c->sf.G, "sfG");
  if (st == DGPYR_OK) st = upload(c, ops.sfGt, &c->sf.Gt, "sfGt");
  if (st == DGPYR_OK) st = upload(c, ops.sfGp, &c->sf.Gp, "sfGp");
  if (st == DGPYR_OK) st = upload(c, ops.sfGb, &c->sf.Gb, "sfGb");
  if (st == DGPYR_OK) st = upload(c, ops.sfGf, &c->sf.Gf, "sfGf");
  if (st == DGPYR_OK) st = upload(c, ops.wc, &c->sf.wc, "sfwc");
  if (st == DGPYR_OK)
    st = c->precision == DGPYR_SPLIT_BF16 ? upload_bf16(c, ops)
         : c->precision == DGPYR_FP32_MFMA ? upload_frags<float>(c, ops)
                                           : upload_frags<double>(c, ops);
  {  // FP64 fragments of the transposed operator
    const double* pd = nullptr;
    if (st == DGPYR_OK && (st = upload(c, frag_rows<double>(ops.V, ops.Nc, ops.Np), &pd, "VrF")) == DGPYR_OK) c->adj.VrF = pd;
    if (st == DGPYR_OK && (st = upload(c, frag_proj<double>(ops.Dr, ops.Nc, ops.Np), &pd, "DrP")) == DGPYR_OK) c->adj.DrP = pd;
    if (st == DGPYR_OK && (st = upload(c, frag_proj<double>(ops.Ds, ops.Nc, ops.Np), &pd, "DsP")) == DGPYR_OK) c->adj.DsP = pd;
    if (st == DGPYR_OK && (st = upload(c, frag_proj<double>(ops.Dt, ops.Nc, ops.Np), &pd, "DtP")) == DGPYR_OK) c->adj.DtP = pd;
    if (st == DGPYR_OK && (st = upload(c, frag_proj<double>(ops.Vf, ops.Nfc, ops.Np), &pd, "LfP")) == DGPYR_OK) c->adj.LfP = pd;
  }
  if (st == DGPYR_OK) st = upload_mesh(c, md);
  if (st == DGPYR_OK) st = alloc(c, (size_t)c->K * c->Nfc * 4 * sizeof(double), &c->T, "trace buffer");
  if (st == DGPYR_OK && (c->reference_kernels || c->unfused))
    st = alloc(c, (size_t)c->K * 4 * c->Np * sizeof(double), &c->vol, "volume buffer");
  return st;
}

// Every device buffer the discrete-adjoint calls use (DGPYR_FLAG_ADJOINT):
// M^-1 Kmat lam, the reverse step's nine state-sized arrays, the adjoint
// traces and the receiver tables at their reserved capacity.
dgpyr_status reserve_adjoint(dgpyr_ctx* c) {
  const size_t state = (size_t)c->K * 4 * c->Np * sizeof(double);
  dgpyr_status st = alloc(c, state, &c->adj_mu, "adjoint scratch");
  if (st == DGPYR_OK) st = alloc(c, 9 * state, &c->adj_work, "adjoint step scratch");
  if (st == DGPYR_OK)
    st = alloc(c, (size_t)c->K * c->Nfc * 4 * sizeof(double), &c->adj_T, "adjoint trace scratch");
  double* re = nullptr;
  double* rp = nullptr;
  if (st == DGPYR_OK)
    st = alloc(c, (size_t)DGPYR_MAX_RESERVED_RECEIVERS * sizeof(int64_t), &re, "receiver elements");
  if (st == DGPYR_OK)
    st = alloc(c, (size_t)DGPYR_MAX_RESERVED_RECEIVERS * c->Np * sizeof(double), &rp,
               "receiver basis values");
  if (st == DGPYR_OK) {
    c->rec_elem = reinterpret_cast<const int64_t*>(re);
    c->rec_phi = rp;
    c->rec_cap = DGPYR_MAX_RESERVED_RECEIVERS;
    c->reserved = true;
  }
  return st;
}

dgpyr_status setup_impl(const dgpyr_mesh* mesh, int32_t N, const dgpyr_opts* opts,
                        const double* dtscale, const int64_t* src_range, dgpyr_ctx** out) {
  if (!out) return fail(DGPYR_E_ARG, "out is null");
  *out = nullptr;
  if (!mesh || !opts) return fail(DGPYR_E_ARG, "mesh or opts is null");
  if (!mesh->xyz || !mesh->e2v || mesh->nverts <= 0 || mesh->nelems <= 0)
    return fail(DGPYR_E_ARG, "mesh arrays must be non-null with positive sizes");
  if (mesh->nelems > (int64_t)0x7fffffff) return fail(DGPYR_E_ARG, "more than 2^31-1 elements");
  if (N < 0 || N > DGPYR_MAX_ORDER) return fail(DGPYR_E_ORDER, "N must be in [0, 8]");
  if (mesh->bc != DGPYR_BC_WALL && mesh->bc != DGPYR_BC_FREE) return fail(DGPYR_E_ARG, "bad bc");
  if (opts->flags & ~(uint32_t)(DGPYR_FLAG_REFERENCE_KERNELS | DGPYR_FLAG_UNFUSED |
                                DGPYR_FLAG_SUM_FACTORIZED | DGPYR_FLAG_ADJOINT |
                                DGPYR_FLAG_WATCHDOG))
    return fail(DGPYR_E_ARG, "unknown flag bits");
  if ((opts->flags & DGPYR_FLAG_SUM_FACTORIZED) &&
      (opts->precision != DGPYR_FP64 || (opts->flags & (DGPYR_FLAG_REFERENCE_KERNELS | DGPYR_FLAG_UNFUSED))))
    return fail(DGPYR_E_UNSUPPORTED, "the sum-factorised kernels are FP64 and fused only");
  if (!(opts->alpha >= 0.0)) return fail(DGPYR_E_ARG, "alpha must be >= 0");
  if (opts->precision != DGPYR_FP64 && opts->precision != DGPYR_FP32_MFMA &&
      opts->precision != DGPYR_SPLIT_BF16)
    return fail(DGPYR_E_ARG, "unknown precision form");
  if (opts->precision == DGPYR_SPLIT_BF16 && (opts->flags & DGPYR_FLAG_UNFUSED))
    return fail(DGPYR_E_UNSUPPORTED, "the split-BF16 form is fused only");
  if ((opts->flags & DGPYR_FLAG_REFERENCE_KERNELS) && opts->precision != DGPYR_FP64)
    return fail(DGPYR_E_UNSUPPORTED, "the reference kernels are FP64 only");

  dgpyr_ctx* c = new (std::nothrow) dgpyr_ctx();
  if (!c) return fail(DGPYR_E_OOM, "host allocation failed");
  char msg[256];
  dgpyr::RefOps ops;
  if (!dgpyr::build_refops(N, ops, msg, sizeof msg)) {
    free_ctx(c);
    return fail(DGPYR_E_STATE, msg);
  }
  dgpyr::MeshData md;
  std::string err;
  int rc = dgpyr::build_mesh(ops, mesh->nverts, mesh->xyz, mesh->nelems, mesh->e2v, mesh->rho,
                             mesh->kappa, md, err);
  if (rc != 0) {
    free_ctx(c);
    return fail((dgpyr_status)rc, err);
  }
  if (mesh->nsources < 0 || (mesh->nsources > 0 && !mesh->sources)) {
    free_ctx(c);
    return fail(DGPYR_E_ARG, "bad source list");
  }
  if (mesh->nsources > 0) {
    rc = dgpyr::locate_sources(ops, mesh->nsources, mesh->sources, src_range, md, err);
    if (rc != 0) {
      free_ctx(c);
      return fail((dgpyr_status)rc, err);
    }
  }
  if (dtscale)
    for (int64_t e = 0; e < md.K; ++e) md.mat[4 * e + 3] = dtscale[e];
  c->mat_host = md.mat;
  c->verts_host = md.verts;
  c->N = N;
  c->Np = ops.Np;
  c->Nc = ops.Nc;
  c->Nfq = ops.Nfq;
  c->Nfc = ops.Nfc;
  c->K = mesh->nelems;
  c->precision = opts->precision;
  c->bc = mesh->bc;
  c->alpha = opts->alpha;
  c->inv_length_max = md.inv_length_max;
  c->inv_length = md.inv_length;
  c->hex_groups = md.hex_groups;
  c->reference_kernels = (opts->flags & DGPYR_FLAG_REFERENCE_KERNELS) != 0;
  c->unfused = (opts->flags & DGPYR_FLAG_UNFUSED) != 0;
  c->sum_factorized = (opts->flags & DGPYR_FLAG_SUM_FACTORIZED) != 0;
  // whole hexahedra per workgroup when the mesh comes in groups of 6 pyramids
  // around a common apex and such a group fits the workgroup's LDS at this N
  c->sf_local = c->sum_factorized && c->hex_groups && dgpyr::sf_local_possible(*c);
  c->mfma_groups = default_groups(N, opts->precision);
  // Operator staging in LDS: measured at 384000 pyramids, N = 4, it speeds the
  // FP32 stage up (2.47 -> 2.29 ms) but slows the FP64 one (3.09 -> 3.44 ms;
  // N = 5 at 196608 pyramids: 3.84 -> 4.64 ms), so it is on for FP32 only.
  c->lds_operators = opts->precision == DGPYR_FP32_MFMA;

  // first device work: the device of the context and its static scratch
  hipError_t ed = hipGetDevice(&c->device);
  dgpyr_status st = ed == hipSuccess ? scratch_for_current_device(c->device)
                                     : hip_fail(ed, "hipGetDevice");
  if (st == DGPYR_OK) st = upload_context(c, ops, md);
  if (st == DGPYR_OK && c->sum_factorized) {
    std::string rmsg;  // LDS, private memory and block size against the device
    st = dgpyr::sf_check_resources(*c, rmsg);
    if (st != DGPYR_OK) st = fail(st, rmsg);
  }
  if (st == DGPYR_OK && (opts->flags & DGPYR_FLAG_ADJOINT)) st = reserve_adjoint(c);
  if (st == DGPYR_OK && (opts->flags & DGPYR_FLAG_WATCHDOG)) {
    const unsigned long long* pw = nullptr;
    st = upload(c, std::vector<unsigned long long>(1, ~0ull), &pw, "watchdog");
    c->watch = const_cast<unsigned long long*>(pw);
  }
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

}  // namespace api
}  // namespace dgpyr

extern "C" {

dgpyr_status dgpyr_setup(const dgpyr_mesh* mesh, int32_t N, const dgpyr_opts* opts, void* stream,
                         dgpyr_ctx** out) {
  (void)stream;
  return setup_impl(mesh, N, opts, nullptr, nullptr, out);
}

dgpyr_status dgpyr_get_info(const dgpyr_ctx* c, dgpyr_info* info) {
  if (dgpyr_status s = check_ctx(c)) return s;
  if (!info) return fail(DGPYR_E_ARG, "info is null");
  info->N = c->N;
  info->Np = c->Np;
  info->Nc = c->Nc;
  info->Nfc = c->Nfc;
  info->nelems = c->K;
  info->state_len = c->K * c->nfields * c->Np;
  info->canon_len = c->K * c->nfields * c->Np;
  info->inv_length_max = c->inv_length_max;
  info->hex_groups = c->hex_groups ? 1 : 0;
  info->precision = c->precision;
  info->device_bytes = c->device_bytes;
  info->groups_per_wave = c->mfma_groups;
  info->nfields = c->nfields;
  return DGPYR_OK;
}

dgpyr_status dgpyr_stable_dt(const dgpyr_ctx* c, double cfl, double* dt) {
  if (dgpyr_status s = check_ctx(c)) return s;
  if (!dt) return fail(DGPYR_E_ARG, "dt is null");
  if (!(cfl > 0.0)) return fail(DGPYR_E_ARG, "cfl must be positive");
  if (!(c->inv_length_max > 0.0)) return fail(DGPYR_E_STATE, "no positive length scale");
  const double CN = 2.0 * (c->N + 1) * (c->N + 3) / 3.0;
  *dt = cfl / (CN * c->inv_length_max);
  return DGPYR_OK;
}

dgpyr_status dgpyr_pack(dgpyr_ctx* c, const double* canon, double* U, void* stream) {
  if (dgpyr_status s = check_ctx(c)) return s;
  if (!canon || !U) return fail(DGPYR_E_ARG, "null array");
  hipError_t e = hipMemcpyAsync(U, canon, (size_t)c->K * c->nfields * c->Np * sizeof(double),
                                hipMemcpyDeviceToDevice, (hipStream_t)stream);
  return e == hipSuccess ? DGPYR_OK : hip_fail(e, "pack");
}

dgpyr_status dgpyr_unpack(dgpyr_ctx* c, const double* U, double* canon, void* stream) {
  if (dgpyr_status s = check_ctx(c)) return s;
  if (!canon || !U) return fail(DGPYR_E_ARG, "null array");
  hipError_t e = hipMemcpyAsync(canon, U, (size_t)c->K * c->nfields * c->Np * sizeof(double),
                                hipMemcpyDeviceToDevice, (hipStream_t)stream);
  return e == hipSuccess ? DGPYR_OK : hip_fail(e, "unpack");
}

dgpyr_status dgpyr_rhs(dgpyr_ctx* c, const double* U, double* dUdt, double t, void* stream) {
  if (dgpyr_status s = check_ctx(c)) return s;
  if (!U || !dUdt) return fail(DGPYR_E_ARG, "null array");
  if ((const double*)dUdt == U) return fail(DGPYR_E_ARG, "U and dUdt must not alias");
  c->mesh.clock = nullptr;
  c->mesh.t_base = t;
  c->mesh.c_stage = 0.0;
  c->mesh.dt_time = 0.0;
  hipError_t e = run_stage(c, 0, U, dUdt, nullptr, 0.0, 0.0, 0.0, (hipStream_t)stream, nullptr);
  return e == hipSuccess ? DGPYR_OK : hip_fail(e, "rhs launch");
}

// NaN/Inf check of the state after step n of the current call.
static hipError_t watch_state(dgpyr_ctx* c, const double* U, int n, hipStream_t s) {
  return dgpyr::launch_nonfinite(U, c->K * c->nfields * c->Np,
                                 (unsigned long long)(c->watch_steps + n), c->watch, s);
}

dgpyr_status dgpyr_watchdog(dgpyr_ctx* c, int64_t* first_bad_step, void* stream) {
  if (dgpyr_status s = check_ctx(c)) return s;
  if (!first_bad_step) return fail(DGPYR_E_ARG, "first_bad_step is null");
  if (!c->watch) return fail(DGPYR_E_STATE, "context set up without DGPYR_FLAG_WATCHDOG");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  unsigned long long v = 0;
  const unsigned long long none = ~0ull;
  e = hipMemcpy(&v, c->watch, sizeof v, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(c->watch, &none, sizeof none, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "watchdog copy");
  c->watch_steps = 0;
  *first_bad_step = v == none ? -1 : (int64_t)v;
  return DGPYR_OK;
}

dgpyr_status dgpyr_step(dgpyr_ctx* c, double* U, double* R, double t0, double dt, int32_t nsteps,
                        void* stream) {
  if (dgpyr_status s = check_ctx(c)) return s;
  if (!U || !R) return fail(DGPYR_E_ARG, "null array");
  if (U == R) return fail(DGPYR_E_ARG, "U and R must not alias");
  if (nsteps < 0) return fail(DGPYR_E_ARG, "nsteps must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = dgpyr::launch_clock(c->clock, 0.0, false, s);
  if (e != hipSuccess) return hip_fail(e, "clock");
  c->mesh.clock = c->clock;
  c->mesh.t_base = t0;
  c->mesh.dt_time = dt;
  for (int n = 0; n < nsteps; ++n) {
    for (int st = 0; st < 5; ++st) {
      c->mesh.c_stage = kRkC.c[st];
      e = run_stage(c, 1, U, U, R, kRkA[st], kRkB[st], dt, s, nullptr);
      if (e != hipSuccess) return hip_fail(e, "step launch");
    }
    e = dgpyr::launch_clock(c->clock, 1.0, true, s);
    if (e != hipSuccess) return hip_fail(e, "clock");
    if (c->watch && (e = watch_state(c, U, n, s)) != hipSuccess) return hip_fail(e, "watchdog");
  }
  c->watch_steps += nsteps;
  return DGPYR_OK;
}

dgpyr_status dgpyr_step_timed(dgpyr_ctx* c, double* U, double* R, double t0, double dt,
                              int32_t nsteps, void* stream, int32_t nk, double* kernel_ms,
                              int64_t* launches) {
  if (dgpyr_status s = check_ctx(c)) return s;
  if (!U || !R) return fail(DGPYR_E_ARG, "null array");
  if (U == R) return fail(DGPYR_E_ARG, "U and R must not alias");
  if (nsteps < 0 || nk < 0 || (nk > 0 && (!kernel_ms || !launches)))
    return fail(DGPYR_E_ARG, "bad nsteps / timing arrays");
  for (int k = 0; k < nk; ++k) {
    kernel_ms[k] = 0.0;
    launches[k] = 0;
  }
  hipStream_t s = (hipStream_t)stream;
  LaunchTimer tm(s, nk, kernel_ms, launches);
  if (tm.err != hipSuccess) return hip_fail(tm.err, "event create");
  hipError_t ec = dgpyr::launch_clock(c->clock, 0.0, false, s);
  if (ec != hipSuccess) return hip_fail(ec, "clock");
  c->mesh.clock = c->clock;
  c->mesh.t_base = t0;
  c->mesh.dt_time = dt;
  for (int n = 0; n < nsteps; ++n) {
    for (int st = 0; st < 5; ++st) {
      c->mesh.c_stage = kRkC.c[st];
      hipError_t e = run_stage(c, 1, U, U, R, kRkA[st], kRkB[st], dt, s, &tm);
      if (e != hipSuccess) return hip_fail(e, "step launch");
    }
    ec = dgpyr::launch_clock(c->clock, 1.0, true, s);
    if (ec != hipSuccess) return hip_fail(ec, "clock");
    if (c->watch && (ec = watch_state(c, U, n, s)) != hipSuccess) return hip_fail(ec, "watchdog");
  }
  c->watch_steps += nsteps;
  tm.drain();
  if (tm.err != hipSuccess) return hip_fail(tm.err, "event timing");
  hipError_t e = hipStreamSynchronize(s);
  return e == hipSuccess ? DGPYR_OK : hip_fail(e, "stream synchronize");
}

dgpyr_status dgpyr_adjoint_rhs(dgpyr_ctx* c, const double* lam, double* out, void* stream) {
  if (dgpyr_status s = check_acoustic(c)) return s;
  if (!lam || !out) return fail(DGPYR_E_ARG, "null array");
  if ((const double*)out == lam) return fail(DGPYR_E_ARG, "lam and out must not alias");
  hipStream_t s = (hipStream_t)stream;
  if (!c->adj_mu) {
    if (dgpyr_status st = alloc(c, (size_t)c->K * 4 * c->Np * sizeof(double), &c->adj_mu,
                                "adjoint scratch"))
      return st;
  }
  hipError_t e = dgpyr::launch_adjoint_scale(*c, lam, c->adj_mu, s);
  if (e == hipSuccess) e = dgpyr::launch_trace_mfma(*c, c->adj_mu, c->T, s);
  if (e == hipSuccess) e = dgpyr::launch_adjoint(*c, c->adj_mu, c->T, out, s);
  return e == hipSuccess ? DGPYR_OK : hip_fail(e, "adjoint launch");
}

dgpyr_status dgpyr_adjoint_rhs_noalloc(dgpyr_ctx* c, const double* lam, double* out,
                                       void* stream) {
  if (dgpyr_status s = check_acoustic(c)) return s;
  if (!lam || !out) return fail(DGPYR_E_ARG, "null array");
  if ((const double*)out == lam) return fail(DGPYR_E_ARG, "lam and out must not alias");
  const size_t need = (size_t)c->K * 4 * c->Np;
  if (need > kScratchDoubles)
    return fail(DGPYR_E_ARG, "state of " + std::to_string(need * sizeof(double)) +
                                 " bytes exceeds the static scratch of " +
                                 std::to_string(DGPYR_NOALLOC_SCRATCH_BYTES) + " bytes");
  double* mu = scratch_ptr(c->device);
  if (!mu) return fail(DGPYR_E_STATE, "static scratch not set up on the context's device");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = dgpyr::launch_adjoint_scale(*c, lam, mu, s);
  if (e == hipSuccess) e = dgpyr::launch_trace_mfma(*c, mu, c->T, s);
  if (e == hipSuccess) e = dgpyr::launch_adjoint(*c, mu, c->T, out, s);
  return e == hipSuccess ? DGPYR_OK : hip_fail(e, "adjoint launch");
}

dgpyr_status dgpyr_set_trace_groups(dgpyr_ctx* c, int32_t groups) {
  if (dgpyr_status s = check_acoustic(c)) return s;
  if (groups != 0 && groups != 1 && groups != 2 && groups != 4)
    return fail(DGPYR_E_ARG, "trace groups must be 0, 1, 2 or 4");
  c->trace_groups = groups;
  return DGPYR_OK;
}

dgpyr_status dgpyr_set_operator_staging(dgpyr_ctx* c, int32_t enable) {
  if (dgpyr_status s = check_acoustic(c)) return s;
  c->lds_operators = enable != 0;
  return DGPYR_OK;
}

dgpyr_status dgpyr_set_groups(dgpyr_ctx* c, int32_t groups) {
  if (dgpyr_status s = check_acoustic(c)) return s;
  if (groups < 0 || groups > 2) return fail(DGPYR_E_ARG, "groups_per_wave must be 0, 1 or 2");
  c->mfma_groups = groups == 0 ? default_groups(c->N, c->precision) : groups;
  return DGPYR_OK;
}

const char* dgpyr_kernel_names(const dgpyr_ctx* c) {
  if (!c) return "";
  return kernel_names(c);
}

dgpyr_status dgpyr_host_reference(int32_t N, int32_t which, double* out, int64_t len,
                                  int64_t* needed) {
  if (N < 0 || N > DGPYR_MAX_ORDER) return fail(DGPYR_E_ORDER, "N must be in [0, 8]");
  if (!needed || len < 0) return fail(DGPYR_E_ARG, "needed is null or len < 0");
  dgpyr::RefOps o;
  char msg[256];
  if (!dgpyr::build_refops(N, o, msg, sizeof msg)) return fail(DGPYR_E_STATE, msg);
  std::vector<double> v;
  switch (which) {
    case 0: v = o.wv; break;
    case 1: v = o.V; break;
    case 2: v = o.Dr; break;
    case 3: v = o.Ds; break;
    case 4: v = o.Dt; break;
    case 5: v = o.Vf; break;
    case 6: v = o.wf; break;
    case 7: v = o.wwc; break;
    case 8:
      for (int r = 0; r < o.Nq1; ++r)
        for (int m = 0; m < o.Nq1; ++m)
          for (int p = 0; p < o.Nq1; ++p) {
            v.push_back(o.xg[p]);
            v.push_back(o.xg[m]);
            v.push_back(o.xc[r]);
          }
      break;
    case 9:
      for (int q = 0; q < o.Nfc; ++q) {
        v.push_back(o.fa[q]);
        v.push_back(o.fb[q]);
        v.push_back(o.fc[q]);
      }
      break;
    case 10: v = o.sfLa; break;
    case 11: v = o.sfDa; break;
    case 12: v = o.sfLe; break;
    case 13: v = o.sfG; break;
    case 14: v = o.sfGt; break;
    case 15: v = o.sfGp; break;
    case 16: v = o.sfGb; break;
    case 17: v = o.sfGf; break;
    default: return fail(DGPYR_E_ARG, "unknown reference array");
  }
  *needed = (int64_t)v.size();
  if (out) std::memcpy(out, v.data(), sizeof(double) * (size_t)std::min<int64_t>(len, *needed));
  return DGPYR_OK;
}

dgpyr_status dgpyr_host_mesh(const dgpyr_mesh* mesh, int32_t N, int32_t* nbr,
                             double* inv_length_max, int32_t* hex_groups) {
  if (!mesh || !mesh->xyz || !mesh->e2v || mesh->nverts <= 0 || mesh->nelems <= 0)
    return fail(DGPYR_E_ARG, "mesh arrays must be non-null with positive sizes");
  if (N < 0 || N > DGPYR_MAX_ORDER) return fail(DGPYR_E_ORDER, "N must be in [0, 8]");
  dgpyr::RefOps ops;
  char msg[256];
  if (!dgpyr::build_refops(N, ops, msg, sizeof msg)) return fail(DGPYR_E_STATE, msg);
  dgpyr::MeshData md;
  std::string err;
  int rc = dgpyr::build_mesh(ops, mesh->nverts, mesh->xyz, mesh->nelems, mesh->e2v, mesh->rho,
                             mesh->kappa, md, err);
  if (rc != 0) return fail((dgpyr_status)rc, err);
  if (nbr)
    for (int64_t e = 0; e < md.K; ++e)
      for (int f = 0; f < 5; ++f) nbr[5 * e + f] = md.conn[(size_t)e * 8 + f];
  if (inv_length_max) *inv_length_max = md.inv_length_max;
  if (hex_groups) *hex_groups = md.hex_groups ? 1 : 0;
  return DGPYR_OK;
}

dgpyr_status dgpyr_host_sources(const dgpyr_mesh* mesh, int32_t N, int64_t* elem, double* abc) {
  if (!mesh || !mesh->xyz || !mesh->e2v || mesh->nverts <= 0 || mesh->nelems <= 0)
    return fail(DGPYR_E_ARG, "mesh arrays must be non-null with positive sizes");
  if (mesh->nsources <= 0 || !mesh->sources) return fail(DGPYR_E_ARG, "no sources");
  if (N < 0 || N > DGPYR_MAX_ORDER) return fail(DGPYR_E_ORDER, "N must be in [0, 8]");
  dgpyr::RefOps ops;
  char msg[256];
  if (!dgpyr::build_refops(N, ops, msg, sizeof msg)) return fail(DGPYR_E_STATE, msg);
  dgpyr::MeshData md;
  std::string err;
  int rc = dgpyr::build_mesh(ops, mesh->nverts, mesh->xyz, mesh->nelems, mesh->e2v, mesh->rho,
                             mesh->kappa, md, err);
  if (rc == 0) rc = dgpyr::locate_sources(ops, mesh->nsources, mesh->sources, nullptr, md, err);
  if (rc != 0) return fail((dgpyr_status)rc, err);
  for (int s = 0; s < mesh->nsources; ++s) {
    if (elem) elem[s] = md.src_elem[(size_t)s];
    if (abc)
      for (int k = 0; k < 3; ++k) abc[3 * s + k] = md.src_abc[(size_t)3 * s + k];
  }
  return DGPYR_OK;
}

dgpyr_status dgpyr_volume_points(dgpyr_ctx* c, double* xyz, double* wJ, void* stream) {
  if (dgpyr_status s = check_ctx(c)) return s;
  if (!xyz) return fail(DGPYR_E_ARG, "xyz is null");
  hipError_t e = dgpyr::launch_points(*c, xyz, wJ, (hipStream_t)stream);
  return e == hipSuccess ? DGPYR_OK : hip_fail(e, "volume points launch");
}

dgpyr_status dgpyr_project(dgpyr_ctx* c, const double* f, double* U, void* stream) {
  if (dgpyr_status s = check_ctx(c)) return s;
  if (!f || !U) return fail(DGPYR_E_ARG, "null array");
  hipError_t e = dgpyr::launch_project(*c, f, U, (hipStream_t)stream);
  return e == hipSuccess ? DGPYR_OK : hip_fail(e, "project launch");
}

dgpyr_status dgpyr_eval(dgpyr_ctx* c, const double* U, double* f, void* stream) {
  if (dgpyr_status s = check_ctx(c)) return s;
  if (!f || !U) return fail(DGPYR_E_ARG, "null array");
  hipError_t e = dgpyr::launch_eval(*c, U, f, (hipStream_t)stream);
  return e == hipSuccess ? DGPYR_OK : hip_fail(e, "eval launch");
}

void dgpyr_destroy(dgpyr_ctx* c) {
  if (!c) return;
  hipDeviceSynchronize();
  free_ctx(c);
}

}  // extern "C"
