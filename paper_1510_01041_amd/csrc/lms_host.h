// Host-side utilities shared by the C-ABI entry points: error reporting,
// per-(device, stream) workspaces, and HIP-event stage timing.
#ifndef LMS_HOST_H
#define LMS_HOST_H
#include <hip/hip_runtime.h>

#include <array>
#include <mutex>
#include <string>

#include "lms.h"

namespace lms_host {

// Records msg as this thread's last error and returns s.
lms_status fail(lms_status s, const std::string& msg);
void clear_error();
const char* last_error();

// A device buffer of at least `bytes` owned by the library, one per
// (device, stream, tag). Growing it first synchronises the stream, since
// queued work may still use the old buffer. Freed by free_workspaces().
lms_status get_workspace(int tag, void* stream, size_t bytes, char** base);
void free_workspaces();
void free_workspace(int tag, void* stream);

// Frees the cached batch plans, buffers and graphs (lms_batched.hip).
void release_batches();

// Autotuned tile choices per (device architecture, path, size class),
// optionally persisted as JSON in the file named by LMS_TUNE_FILE.
bool get_tuning(int path, int size_class, lms_tuning* t);
void set_tuning(int path, int size_class, const lms_tuning& t);
void clear_tuning();
int size_class(int n);  // next power of two >= n (>= 64)

// Seed-network inference (lms_net.hip): device bytes of its scratch for B
// sets, and the launches (frame, pooled features over many workgroups, head
// and slope) into d_theta (and the raw outputs into d_out if not NULL).
// d_offsets NULL: one set of max_set points at d_xy (B = 1).
size_t net_infer_bytes(int64_t B);
lms_status net_infer_enqueue(const float* d_params, const double* d_xy, const int64_t* d_offsets,
                             int64_t B, int64_t max_set, int max_points, double* d_theta,
                             float* d_out, void* scratch, hipStream_t s);

// Compute units of the current device (queried once).
int num_cu();

// HIP events around the stages of one solve, kept while profiling is on.
struct StageEvents {
  std::array<hipEvent_t, LMS_NSTAGES + 1> ev{};
  bool on = false;
  hipStream_t s = nullptr;
  int next = 0;
  void start(hipStream_t stream);
  void mark();
  void finish();
};
void profile_begin();
int64_t profile_end(double* ms);

}  // namespace lms_host

#endif
