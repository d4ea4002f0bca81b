// Batches of independent problems: many meshes of different sizes and orders
// advanced together.  Problems are grouped by (N, boundary condition); the
// meshes of a group are concatenated into one context (no face is shared
// between problems, so the concatenation is exact), each element carrying
// its own problem's time step in its material row.  One LSRK step of every
// group is captured once into a HIP graph -- the groups on streams of their
// own between a fork and a join, so independent groups run concurrently --
// and replayed on the caller's stream; a per-group autotuner picks the kernels
// and work shape of each order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "context.hpp"
#include "dgpyr.h"
#include "internal.hpp"

using namespace dgpyr::api;

struct dgpyr_batch {
  struct Group {
    int N = 0, bc = 0;
    dgpyr_ctx* ctx = nullptr;
    int64_t state_off = 0, state_len = 0;
    std::vector<int> problems;
  };
  std::vector<Group> groups;
  std::vector<dgpyr_batch_slot> slots;
  int64_t state_len = 0;
  hipStream_t cap = nullptr;  // private stream used only for graph capture
  // one stream and one event per group: the captured step forks from cap
  // into the groups and joins back, so independent groups run concurrently
  std::vector<hipStream_t> gs;
  std::vector<hipEvent_t> gev;
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const double* gU = nullptr;  // state arrays the captured graph uses
  const double* gR = nullptr;
};

namespace {

void drop_graph(dgpyr_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->gU = b->gR = nullptr;
}

void free_batch(dgpyr_batch* b) {
  if (!b) return;
  drop_graph(b);
  for (auto& g : b->groups) free_ctx(g.ctx);
  for (hipEvent_t ev : b->gev)
    if (ev) hipEventDestroy(ev);
  for (hipStream_t st : b->gs)
    if (st) hipStreamDestroy(st);
  if (b->fork) hipEventDestroy(b->fork);
  if (b->cap) hipStreamDestroy(b->cap);
  delete b;
}

// One LSRK step of group g on stream s, the time step of each element taken
// from its material row (dt = 1 times the per-element scale).
hipError_t enqueue_group_step(dgpyr_batch::Group& g, double* U, double* R, hipStream_t s) {
  dgpyr_ctx* c = g.ctx;
  double* Ug = U + g.state_off;
  double* Rg = R + g.state_off;
  c->mesh.clock = c->clock;
  c->mesh.t_base = 0.0;
  c->mesh.dt_time = 1.0;
  for (int st = 0; st < 5; ++st) {
    c->mesh.c_stage = kRkC.c[st];
    hipError_t e = run_stage(c, 1, Ug, Ug, Rg, kRkA[st], kRkB[st], 1.0, s, nullptr);
    if (e != hipSuccess) return e;
  }
  return dgpyr::launch_clock(c->clock, 1.0, true, s);
}

// One step of every group, forked from stream s onto the groups' streams and
// joined back (groups share no data, so they may run concurrently).
hipError_t enqueue_step(dgpyr_batch* b, double* U, double* R, hipStream_t s) {
  hipError_t e = hipEventRecord(b->fork, s);
  for (size_t g = 0; g < b->groups.size() && e == hipSuccess; ++g) {
    e = hipStreamWaitEvent(b->gs[g], b->fork, 0);
    if (e == hipSuccess) e = enqueue_group_step(b->groups[g], U, R, b->gs[g]);
    if (e == hipSuccess) e = hipEventRecord(b->gev[g], b->gs[g]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, b->gev[g], 0);
  }
  return e;
}

dgpyr_status capture(dgpyr_batch* b, double* U, double* R) {
  drop_graph(b);
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "begin capture");
  hipError_t el = enqueue_step(b, U, R, b->cap);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap, &g);
  if (el != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return hip_fail(el, "captured launch");
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return hip_fail(e, "graph instantiate");
  }
  b->graph = g;
  b->exec = x;
  b->gU = U;
  b->gR = R;
  return DGPYR_OK;
}

dgpyr_status check_batch(const dgpyr_batch* b) {
  if (!b) return fail(DGPYR_E_ARG, "null batch");
  return DGPYR_OK;
}

}  // namespace

extern "C" {

dgpyr_status dgpyr_batch_setup(const dgpyr_mesh* meshes, const int32_t* orders,
                               const double* dts, double cfl, int32_t nproblems,
                               const dgpyr_opts* opts, dgpyr_batch** out) {
  if (!out) return fail(DGPYR_E_ARG, "out is null");
  *out = nullptr;
  if (!meshes || !orders || !opts || nproblems <= 0)
    return fail(DGPYR_E_ARG, "meshes, orders and opts must be non-null, nproblems > 0");
  if (!dts && !(cfl > 0)) return fail(DGPYR_E_ARG, "give dts or a positive cfl");
  for (int i = 0; i < nproblems; ++i) {
    const dgpyr_mesh& m = meshes[i];
    if (!m.xyz || !m.e2v || m.nverts <= 0 || m.nelems <= 0)
      return fail(DGPYR_E_ARG, "problem " + std::to_string(i) + ": empty mesh");
    if (orders[i] < 0 || orders[i] > DGPYR_MAX_ORDER)
      return fail(DGPYR_E_ORDER, "problem " + std::to_string(i) + ": N must be in [0, 8]");
    if (m.nsources < 0 || (m.nsources > 0 && !m.sources))
      return fail(DGPYR_E_ARG, "problem " + std::to_string(i) + ": bad source list");
    if (dts && !(dts[i] > 0)) return fail(DGPYR_E_ARG, "problem " + std::to_string(i) + ": dt <= 0");
  }
  dgpyr_batch* b = new (std::nothrow) dgpyr_batch();
  if (!b) return fail(DGPYR_E_OOM, "host allocation failed");
  b->slots.resize((size_t)nproblems);

  // groups keyed by (N, bc), problems in input order inside a group
  std::map<std::pair<int, int>, int> key;
  for (int i = 0; i < nproblems; ++i) {
    const auto k = std::make_pair((int)orders[i], (int)meshes[i].bc);
    auto it = key.find(k);
    if (it == key.end()) it = key.emplace(k, 0).first;
  }
  int gi = 0;
  for (auto& kv : key) {
    kv.second = gi++;
    dgpyr_batch::Group g;
    g.N = kv.first.first;
    g.bc = kv.first.second;
    b->groups.push_back(g);
  }
  for (int i = 0; i < nproblems; ++i)
    b->groups[(size_t)key[std::make_pair((int)orders[i], (int)meshes[i].bc)]].problems.push_back(i);

  int64_t state_off = 0;
  for (size_t gix = 0; gix < b->groups.size(); ++gix) {
    auto& g = b->groups[gix];
    // concatenated mesh of the group
    std::vector<double> xyz, rho, kappa, src;
    std::vector<int64_t> e2v, range;
    int64_t voff = 0, eoff = 0;
    int nsrc = 0;
    for (int i : g.problems) {
      const dgpyr_mesh& m = meshes[i];
      xyz.insert(xyz.end(), m.xyz, m.xyz + 3 * m.nverts);
      for (int64_t j = 0; j < 5 * m.nelems; ++j) {
        const int64_t v = m.e2v[j];
        if (v < 0 || v >= m.nverts) {
          free_batch(b);
          return fail(DGPYR_E_ARG, "problem " + std::to_string(i) + ": vertex index out of range");
        }
        e2v.push_back(v + voff);
      }
      for (int64_t e = 0; e < m.nelems; ++e) {
        rho.push_back(m.rho ? m.rho[e] : 1.0);
        kappa.push_back(m.kappa ? m.kappa[e] : 1.0);
      }
      for (int s = 0; s < m.nsources; ++s) {
        src.insert(src.end(), m.sources + 6 * s, m.sources + 6 * s + 6);
        range.push_back(eoff);
        range.push_back(eoff + m.nelems);
      }
      nsrc += m.nsources;
      auto& sl = b->slots[(size_t)i];
      sl.group = (int32_t)gix;
      sl.N = g.N;
      sl.Np = (g.N + 1) * (g.N + 2) * (2 * g.N + 3) / 6;
      sl.nelems = m.nelems;
      sl.elem_offset = eoff;
      voff += m.nverts;
      eoff += m.nelems;
    }
    dgpyr_mesh merged{};
    merged.nverts = voff;
    merged.xyz = xyz.data();
    merged.nelems = eoff;
    merged.e2v = e2v.data();
    merged.rho = rho.data();
    merged.kappa = kappa.data();
    merged.bc = g.bc;
    merged.nsources = nsrc;
    merged.sources = nsrc ? src.data() : nullptr;
    dgpyr_status st = setup_impl(&merged, g.N, opts, nullptr, nsrc ? range.data() : nullptr, &g.ctx);
    if (st != DGPYR_OK) {
      free_batch(b);
      return st;
    }
    // per-problem time steps into the material rows
    dgpyr_ctx* c = g.ctx;
    const double CN = 2.0 * (g.N + 1) * (g.N + 3) / 3.0;
    for (int i : g.problems) {
      auto& sl = b->slots[(size_t)i];
      double il = 0.0;
      for (int64_t e = 0; e < sl.nelems; ++e)
        il = std::max(il, c->inv_length[(size_t)(sl.elem_offset + e)]);
      sl.inv_length_max = il;
      sl.dt = dts ? dts[i] : cfl / (CN * il);
      for (int64_t e = 0; e < sl.nelems; ++e) c->mat_host[(size_t)(4 * (sl.elem_offset + e) + 3)] = sl.dt;
    }
    hipError_t he = hipMemcpy(const_cast<double*>(c->mesh.mat), c->mat_host.data(),
                              c->mat_host.size() * sizeof(double), hipMemcpyHostToDevice);
    if (he != hipSuccess) {
      free_batch(b);
      return hip_fail(he, "upload time steps");
    }
    g.state_off = state_off;
    g.state_len = c->K * 4 * c->Np;
    for (int i : g.problems) {
      auto& sl = b->slots[(size_t)i];
      sl.offset = state_off + sl.elem_offset * 4 * sl.Np;
      sl.len = sl.nelems * 4 * sl.Np;
    }
    state_off += g.state_len;
  }
  b->state_len = state_off;
  hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  b->gs.assign(b->groups.size(), nullptr);
  b->gev.assign(b->groups.size(), nullptr);
  for (size_t g = 0; g < b->groups.size() && e == hipSuccess; ++g) {
    e = hipStreamCreateWithFlags(&b->gs[g], hipStreamNonBlocking);  // default priority
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->gev[g], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    free_batch(b);
    return hip_fail(e, "capture streams");
  }
  *out = b;
  return DGPYR_OK;
}

dgpyr_status dgpyr_batch_info(const dgpyr_batch* b, int64_t* state_len, int32_t* ngroups) {
  if (dgpyr_status s = check_batch(b)) return s;
  if (state_len) *state_len = b->state_len;
  if (ngroups) *ngroups = (int32_t)b->groups.size();
  return DGPYR_OK;
}

dgpyr_status dgpyr_batch_problem(const dgpyr_batch* b, int32_t i, dgpyr_batch_slot* slot) {
  if (dgpyr_status s = check_batch(b)) return s;
  if (!slot || i < 0 || i >= (int32_t)b->slots.size()) return fail(DGPYR_E_ARG, "bad problem index");
  *slot = b->slots[(size_t)i];
  return DGPYR_OK;
}

dgpyr_status dgpyr_batch_group(dgpyr_batch* b, int32_t g, dgpyr_ctx** ctx, int64_t* state_offset) {
  if (dgpyr_status s = check_batch(b)) return s;
  if (!ctx || g < 0 || g >= (int32_t)b->groups.size()) return fail(DGPYR_E_ARG, "bad group index");
  *ctx = b->groups[(size_t)g].ctx;
  if (state_offset) *state_offset = b->groups[(size_t)g].state_off;
  return DGPYR_OK;
}

dgpyr_status dgpyr_batch_step(dgpyr_batch* b, double* U, double* R, int64_t step0, int32_t nsteps,
                              void* stream) {
  if (dgpyr_status s = check_batch(b)) return s;
  if (!U || !R) return fail(DGPYR_E_ARG, "null array");
  if (U == R) return fail(DGPYR_E_ARG, "U and R must not alias");
  if (nsteps < 0 || step0 < 0) return fail(DGPYR_E_ARG, "nsteps and step0 must be >= 0");
  if (nsteps == 0) return DGPYR_OK;
  hipStream_t s = (hipStream_t)stream;
  if (!b->exec || b->gU != U || b->gR != R) {
    if (dgpyr_status st = capture(b, U, R)) return st;
  }
  for (auto& g : b->groups) {
    hipError_t e = dgpyr::launch_clock(g.ctx->clock, (double)step0, false, s);
    if (e != hipSuccess) return hip_fail(e, "clock");
  }
  for (int n = 0; n < nsteps; ++n) {
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
  }
  return DGPYR_OK;
}

dgpyr_status dgpyr_batch_tune(dgpyr_batch* b, double* Us, double* Rs, int32_t nsteps, void* stream,
                              int32_t* chosen) {
  if (dgpyr_status s = check_batch(b)) return s;
  if (!Us || !Rs) return fail(DGPYR_E_ARG, "null scratch array");
  if (Us == Rs) return fail(DGPYR_E_ARG, "U and R must not alias");
  if (nsteps <= 0) return fail(DGPYR_E_ARG, "nsteps must be > 0");
  hipStream_t s = (hipStream_t)stream;
  drop_graph(b);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  dgpyr_status st = e == hipSuccess ? DGPYR_OK : hip_fail(e, "event create");
  for (size_t gix = 0; st == DGPYR_OK && gix < b->groups.size(); ++gix) {
    dgpyr_ctx* c = b->groups[gix].ctx;
    const bool tunable = !c->reference_kernels && !c->unfused && c->precision != DGPYR_SPLIT_BF16;
    if (!tunable) {
      if (chosen) chosen[gix] = 0;
      continue;
    }
    // candidate work shapes: matrix-core stage with 1 or 2 element groups per
    // wave times trace kernel with 1, 2 or 4 (code 10 tg + gw), and for FP64
    // the sum-factorised kernels (code 100) where their resources fit
    std::vector<int> cand;
    for (int tg : {1, 2, 4})
      for (int gw : {1, 2}) cand.push_back(10 * tg + gw);
    const bool sf0 = c->sum_factorized, sfl0 = c->sf_local;
    if (c->precision == DGPYR_FP64) {
      c->sum_factorized = true;
      c->sf_local = c->hex_groups && dgpyr::sf_local_possible(*c);
      std::string msg;
      if (dgpyr::sf_check_resources(*c, msg) == DGPYR_OK) cand.push_back(100);
    }
    auto apply = [&](int code) {
      c->sum_factorized = code == 100;
      c->sf_local = c->sum_factorized && c->hex_groups && dgpyr::sf_local_possible(*c);
      if (code != 100) {
        c->mfma_groups = code % 10;
        c->trace_groups = code / 10;
      }
    };
    // the caller's scratch, cleared: the timing does not depend on values
    double* U = Us + b->groups[gix].state_off;
    double* R = Rs + b->groups[gix].state_off;
    e = dgpyr::launch_fill(U, b->groups[gix].state_len, 0.0, s);
    if (e == hipSuccess) e = dgpyr::launch_fill(R, b->groups[gix].state_len, 0.0, s);
    float best = 0.f;
    int pick = 0;
    for (int code : cand) {
      if (e != hipSuccess) break;
      apply(code);
      c->mesh.clock = c->clock;
      for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // warm-up, then timed
        if (rep == 1) e = hipEventRecord(e0, s);
        for (int n = 0; n < nsteps && e == hipSuccess; ++n)
          for (int k = 0; k < 5 && e == hipSuccess; ++k)
            e = run_stage(c, 1, U, U, R, kRkA[k], kRkB[k], 1.0, s, nullptr);
      }
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e == hipSuccess && (pick == 0 || ms < best)) {
        best = ms;
        pick = code;
      }
    }
    if (pick) {
      apply(pick);
    } else {
      c->sum_factorized = sf0;
      c->sf_local = sfl0;
    }
    if (chosen) chosen[gix] = pick;
    if (e != hipSuccess) st = hip_fail(e, "tune");
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  return st;
}

void dgpyr_batch_destroy(dgpyr_batch* b) { free_batch(b); }

}  // extern "C"
