// Internal runtime state of the MAGPIE C ABI shared by the host sources of
// the library: error reporting, device allocation helpers and the
// reconstruction context.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/magpie.h"
#include "kernels.h"

namespace mgrt {

inline thread_local std::string g_last_error;

inline int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define MG_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(MAGPIE_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

inline bool valid_m(int m) { return m == 8 || m == 16 || m == 32 || m == 64 || m == 128; }

inline int ilog2(int m) {
  int l = 0;
  while ((1 << l) < m) ++l;
  return l;
}

template <typename T>
inline int dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return MAGPIE_OK;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(MAGPIE_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  return MAGPIE_OK;
}

template <typename T>
inline void dev_free(T*& p) {
  if (p) hipFree((void*)p);
  p = nullptr;
}

inline uint64_t splitmix64_next(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline void fisher_yates(uint64_t seed, uint64_t epoch, int n, int32_t* out) {
  for (int i = 0; i < n; ++i) out[i] = i;
  uint64_t st = seed ^ epoch;
  for (int i = n - 1; i > 0; --i) {
    const uint64_t j = splitmix64_next(st) % (uint64_t)(i + 1);
    std::swap(out[i], out[(size_t)j]);
  }
}

}  // namespace mgrt

struct magpie_ctx {
  int device = 0;
  int n_cu = 256;   // compute units of the device
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int nr = 0, nc = 0, m = 0, L = 1;
  int rb = 0;    // FFT plan of the step kernel (threads per 1-D transform)
  int th = 8;    // accumulate tile height
  double alpha = 0.0;
  uint32_t flags = 0;
  double beta = 0.0;
  bool u_given = false;
  int n_pos = 0;
  bool has_probe = false, has_pos = false, has_data = false;
  uint64_t epoch_index = 0;

  // device buffers
  float2* z = nullptr;
  float2* qf = nullptr;
  float4* qtab = nullptr;   // (Re Q, Im Q, u0, 0) in the current plan's thread order
  float2* qspec = nullptr;  // F(Q) (computed in FP64) in the current plan's spectral thread order
  double2* spec_tmp = nullptr;   // m*m + m scratch: its row transforms, then the rows' sums of |Q|
  double2* q64 = nullptr;
  double* u0 = nullptr;
  double* w0 = nullptr;
  float* w0f = nullptr;
  float* u0f = nullptr;
  double* lvl = nullptr;
  double2* scr_q = nullptr;
  double* scr_u = nullptr;
  int* flag = nullptr;
  double* red = nullptr;

  int2* offs = nullptr;
  float* sqrtd = nullptr;
  double* phi_step = nullptr;   // per position, reduced on demand
  double* phi_obj = nullptr;
  double* gnorm = nullptr;
  double* step_part = nullptr;  // per-wave partials [N][MAX_WAVES]
  double* obj_part = nullptr;
  double* gn_part = nullptr;
  int lvl_a_off = 0;
  int* tile_ptr = nullptr;
  int4* tile_ent = nullptr;
  int tiles_x = 0, tiles_y = 0;
  int box_x0 = 0, box_y0 = 0, box_nx = 0, box_ny = 0;   // tiles some window reaches
  int scan_r0 = 0, scan_r1 = 0;  // first and last object row some window covers
  std::vector<int32_t> h_offs;

  float2* stage = nullptr;
  size_t stage_cap = 0;  // in float2
  float2* phase = nullptr;  // eq. (3.2) phase store [n_pos][m][m], natural order (flag MAGPIE_PHASE_RECYCLE)
  size_t phase_cap = 0;     // in float2
  float2* pnum = nullptr;   // probe step partials (allocated with the staging when the flag is on)
  float* pden = nullptr;
  float* pmax = nullptr;
  double* pacc = nullptr;   // probe step: per-chunk partial sums (mg::probe_scratch_doubles)
  size_t pcap = 0;
  int4* posrec = nullptr;  // [E][N] (k, row, col, 0) in processing order
  int4* posx = nullptr;    // [E][N] the same records in workgroup order, (k, row, col, slot)
  int* inv = nullptr;    // [E][N] position -> index in its epoch's permutation
  size_t perm_cap = 0;   // entries per array
  // pinned host records in two slots (filled while the GPU runs the other one)
  int32_t* h_pin = nullptr;
  size_t h_pin_cap = 0;  // ints
  size_t pin_width = 0;  // epochs per slot of the last fill
  hipEvent_t pin_done[2] = {nullptr, nullptr};
  bool pin_pending[2] = {false, false};
  // round descriptors of multi-context chunks led by this context (two slots)
  void* mdesc_host[2] = {nullptr, nullptr};
  unsigned char* mdesc_dev[2] = {nullptr, nullptr};
  size_t mdesc_cap[2] = {0, 0};
  hipEvent_t mdesc_done[2] = {nullptr, nullptr};
  bool mdesc_pending[2] = {false, false};
  // work-queue counters of multi-context runs led by this context (per plan
  // partition: done per member, head; then one abort flag for the run)
  int* qctr = nullptr;
  size_t qctr_cap = 0;   // ints
  std::vector<int32_t> h_perm;   // host scratch: one epoch's permutation
  std::vector<int> h_seen;       // host scratch: permutation check
  std::vector<int> h_cnt, h_sorted;   // host scratch: a minibatch's windows bucketed by cell

  // optional per-launch timing
  bool timing = false;
  struct Timed {
    hipEvent_t a, b;
    int kind;   // 0 = step kernel, 1 = accumulate kernel
    int count;  // positions (step kernel)
  };
  std::vector<hipEvent_t> ev_pool;
  std::vector<Timed> timed;

  // captured epoch graph (replayed once per epoch); the epoch index is read
  // by the kernels from epoch_ctr, which the graph's last node advances
  hipGraphExec_t gexec = nullptr;
  int g_batch = 0;
  const void* g_key[4] = {nullptr, nullptr, nullptr, nullptr};  // buffers it was built on
  int* epoch_ctr = nullptr;
  int g_rb = 0, g_th = 0;

  // learned-start scratch (allocated on first use, grown as needed)
  float* lrn_sd = nullptr;       // sqrt(d) in natural order
  size_t lrn_sd_cap = 0;
  double4* lrn_stats = nullptr;  // per-position statistics
  size_t lrn_stats_cap = 0;
  double* lrn_fine = nullptr;    // full-resolution map, 3 channels
  size_t lrn_fine_cap = 0;
  float* lrn_map = nullptr;      // pooled map
  size_t lrn_map_cap = 0;
  double* lrn_q = nullptr;       // ||Q||_2
  float2* lrn_one = nullptr;     // the value 1 + 0i (flat start)
};

namespace mgrt {

inline int set_dev(magpie_ctx* c) {
  MG_HIP(hipSetDevice(c->device));
  return MAGPIE_OK;
}

// Per-epoch device buffers of the launch loop: staging [B][m][m], position
// records (k, row, col, 0) [E][N] in processing order, inverse permutations [E][N].
struct EpochBuffers {
  float2* stage;
  const int4* posrec;
  const int* inv;
  const int4* posx;   // nullable: records in workgroup order (step launches read them if given)
};

// noalloc.hip: resolves the device address of the no-allocation entry point's
// scratch array on `device` (current), once per device.
int noalloc_init_device(int device);

// capi.cpp: launches prepared epochs on the given buffers (see there).
int launch_epochs(magpie_ctx* c, int n_epochs, int B, int batches_per_epoch, bool allow_graph,
                  const EpochBuffers& buf);

inline int read_flag(magpie_ctx* c, int* out) {
  int h = 0;
  MG_HIP(hipMemcpyAsync(&h, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  MG_HIP(hipStreamSynchronize(c->stream));
  *out = h;
  return MAGPIE_OK;
}

}  // namespace mgrt
