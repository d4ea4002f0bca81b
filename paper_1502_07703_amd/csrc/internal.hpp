// Library-internal entry points shared by api.hip (single problems) and
// batch.hip (batches of independent problems).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "context.hpp"
#include "dgpyr.h"

namespace dgpyr {
namespace api {

// Records msg as the thread's last error and returns s.
dgpyr_status fail(dgpyr_status s, const std::string& msg);
dgpyr_status hip_fail(hipError_t e, const char* what);
dgpyr_status check_ctx(const dgpyr_ctx* c);
// check_ctx, and E_UNSUPPORTED for contexts of another equation than acoustics.
dgpyr_status check_acoustic(const dgpyr_ctx* c);

// Carpenter-Kennedy RK(5,4) 2N-storage coefficients and the stage times c_s.
extern const double kRkA[5];
extern const double kRkB[5];
struct StageTimes {
  double c[5];
  StageTimes();
};
extern const StageTimes kRkC;

struct LaunchTimer;

// One LSRK stage (mode 1) or right-hand side (mode 0) on stream s.
hipError_t run_stage(dgpyr_ctx* c, int mode, const double* U, double* out, double* R, double ra,
                     double rb, double dt, hipStream_t s, LaunchTimer* tm);

// Context setup; dtscale ([K], optional) scales the time step per element,
// src_range ([nsources][2], optional) limits each source's element search.
dgpyr_status setup_impl(const dgpyr_mesh* mesh, int32_t N, const dgpyr_opts* opts,
                        const double* dtscale, const int64_t* src_range, dgpyr_ctx** out);

// Uploads reference operators, fragments, per-element data and the trace
// buffer of a context whose sizes, physics and precision are set.
dgpyr_status upload_context(dgpyr_ctx* c, const dgpyr::RefOps& ops, const dgpyr::MeshData& md);

// Device allocation owned by the context (freed with it).
dgpyr_status alloc(dgpyr_ctx* c, size_t bytes, double** out, const char* what);

// Releases a context and its device memory.
void free_ctx(dgpyr_ctx* c);

}  // namespace api
}  // namespace dgpyr
