// Launch wrappers of the gfx950 kernels (plain C++ signatures, no HIP types
// beyond the stream) used by the host runtime in capi.cpp.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mg {

enum StepMode { MODE_STEP = 0, MODE_OBJECTIVE = 1, MODE_FORWARD = 2 };
// (internal) MODE_STEP with the eq. (3.2) phase store, chosen by launch_step when StepArgs::phase is set
constexpr int MODE_STEP_PR = 3;

constexpr int MAX_WAVES = 16;   // per-position partial sums (one per wave of a workgroup)

// The in-wave V-cycle's constant block (doubles), laid out for LDS: A_1..A_{L-1}
// at level-1 resolution, then V_1..V_{L-2} at their own resolutions; every row of
// a grid of side s is padded to s + CST_PAD doubles, so that the rows the lanes of
// one LDS access read fall in different banks.
constexpr int CST_PAD = 2;
__host__ __device__ constexpr int cst_count(int M, int L) {
  int n = (L - 1) * (M / 2) * (M / 2 + CST_PAD);
  for (int l = 1; l <= L - 2; ++l) n += (M >> l) * ((M >> l) + CST_PAD);
  return n;
}
__host__ __device__ constexpr int cst_v_off(int M, int L, int l) {
  int n = (L - 1) * (M / 2) * (M / 2 + CST_PAD);
  for (int j = 1; j < l; ++j) n += (M >> j) * ((M >> j) + CST_PAD);
  return n;
}

// Arguments of the per-position kernel (one workgroup per scan position).
struct StepArgs {
  const float2* z;        // object [n_rows][n_cols]
  int n_rows, n_cols;
  const float2* q;        // probe FP32 [m][m]
  const float* sqrtd;     // sqrt(d) in kernel order [N][m*m]
  const int2* offs;       // (row, col) per position [N]
  const int4* pos;        // MODE_STEP: (k, row, col, 0) of the positions handled, one per workgroup
  const int4* posx;       // MODE_STEP, nullable: the same records in workgroup order, .w = the slot
                          // (index in pos) the workgroup handles; NULL: workgroup i handles slot i
  const int* perm;        // other modes: positions handled; NULL = identity
  const int* epoch;       // nullable: perm is advanced by (*epoch) * epoch_stride (graph replays)
  int epoch_stride;
  int count;              // number of workgroups / positions
  float2* stage;          // MODE_STEP: c_k = w0 * dz_k, natural order [count][m][m]
  const float* u0f;       // fine-grid u [m][m]
  const float4* qtab;     // probe table in the plan's thread order [n1][tid], pixel (RB*n1 + g, col): m <= 64
                          // (Re Q, Im Q, u0, 0) per entry; m = 128 m*m float2 Q, then m*m float u0
  const float2* qspec;    // F(Q) of the FP32 probe, computed in FP64, in the order the forward transform
                          // leaves the spectrum [j][tid] (thread (ky, g), j = c*RB + k2: kx = g*CB + c + RA*k2)
  const double* lvl;      // coarse-level constants (V, rho, r per level), then A_l
  int lvl_a_off;          // offset in lvl of the in-wave V-cycle block (cst_count(m, L) doubles)
  int levels;             // number of grids L
  double* phi_part;       // per-wave partials of Phi_k [N][MAX_WAVES] (nullable)
  double* gn_part;        // MODE_OBJECTIVE: per-wave partials of ||grad_k||^2 [N][MAX_WAVES]
  float* d_out;           // MODE_FORWARD: |F(Q z_k)|^2 natural order [N][m][m]
  float2* probe_num;      // probe step: conj(z_k)(R_k - Q z_k) per position [count][m][m] (nullable)
  float* probe_den;       // probe step: |z_k|^2 per position [count][m][m]
  float* probe_max;       // probe step: per-wave max |z_k|^2 [count][MAX_WAVES]
  float2* phase;          // MODE_STEP, nullable: eq. (3.2) phase store [N][m][m] natural order
  int stage_wt;           // MODE_STEP: store the staged updates with device scope (written through
                          // L2): faster when the launch is one workgroup per CU, slower for large launches
};

struct AccumArgs {
  float2* z;              // object, updated in place
  int n_rows, n_cols, m;
  int tiles_x;            // number of tile columns of the object (ACC_TILE_W wide)
  int box_x0, box_y0;     // first tile column / row of the box of tiles any window reaches
  int box_nx;             // tile columns of that box; workgroup b takes box tile b (row-major)
  int n_tiles;            // tiles of the box (= workgroups)
  const int* tile_ptr;    // CSR over all tiles: positions overlapping each tile, ascending
  const int4* tile_ent;   // (k, row, col, 0) of each overlapping position
  const int4* pos;        // nullable: this minibatch's records (k, row, col, 0), `count` of them in processing
                          // order, screened directly (sums in that order); NULL: the static lists with inv
  int count;
  const int* inv;         // position -> index in this epoch's permutation
  const int* epoch;       // nullable: inv is advanced by (*epoch) * epoch_stride (graph replays)
  int epoch_stride;
  int batch_index, batch; // minibatch t and size B
  const float2* stage;    // [B][m][m]
  const int2* offs;
  const float* w0f;       // u + |Q|^2 [m][m], FP32 copy
};

constexpr int ACC_TILE_W = 32;   // accumulation tile width (two rows per wave)
// one pixel per thread: a 32 x TH tile takes 32 TH threads (TH / 2 waves)
constexpr int acc_threads(int th) { return ACC_TILE_W * th; }
// minibatches of at most this many positions are screened from their own records
constexpr int ACC_SCAN_MAX = 256;

// FFT plans (m, rb): rb threads per 1-D transform.  plans_for lists the
// compiled plans of m, default first.
bool plan_valid(int m, int rb);
int default_plan(int m);
int plans_for(int m, int* rbs, int cap);
bool tile_valid(int th);                    // accumulate tile heights: 8, 16, 32
int step_threads(int m, int rb);            // workgroup size of the per-position kernel
int step_waves(int m, int rb);
size_t step_lds_bytes(int m, int rb);       // dynamic LDS of the per-position kernel

hipError_t init_twiddles(hipStream_t s);
// ev0/ev1 (nullable): events the dispatch itself records at kernel start and end
hipError_t launch_step(int m, int rb, int mode, const StepArgs& a, hipStream_t s, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
hipError_t launch_accumulate(const AccumArgs& a, int th, int n_tiles, hipStream_t s, hipEvent_t ev0 = nullptr,
                             hipEvent_t ev1 = nullptr);
// One launch over several contexts: descriptor j describes context j for this
// round; prefix (device, n_ctx + 1 ints) holds the running totals of the
// contexts' positions (step) or tiles (accumulation), prefix[0] = 0 and
// prefix[n_ctx] = total = the number of workgroups (contexts with none: idle).
hipError_t launch_step_multi(int m, int rb, const StepArgs* descs, const int* prefix, int n_ctx, int total,
                             hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_accumulate_multi(int th, const AccumArgs* descs, const int* prefix, int n_ctx, int total,
                                   hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Work-queue launch over the rounds of a chunk for the members of one FFT plan
// (m, rb): in queue order, group g = (2 r + phase) n_members + j holds the step
// items (phase 0: one per position of member j's round-r minibatch) or the tile
// items (phase 1: one per tile of member j's box at tile height qtile_rows(m, rb))
// of member j in round r, items gpre[g] .. gpre[g + 1] - 1.  A group's items wait
// until done[j + n_members] (tiles finished, for steps) or done[j] (steps
// finished, for tiles) reaches wait[g].  done, head: zero before the launch.
// Each done counter is split into QSLOTS slots QSLOT_STRIDE ints apart (an item
// adds to slot b mod QSLOTS, a wait sums the slots): device-scope atomics on one
// address serialise, and a whole minibatch's items finish at about the same time.
constexpr int QSLOTS = 16, QSLOT_STRIDE = 32;
constexpr size_t queue_counter_ints(int n_members) {
  return ((size_t)2 * n_members * QSLOTS + 1) * QSLOT_STRIDE;   // done slots, then head
}
struct QueueArgs {
  const StepArgs* sdesc;    // [rounds][n_members]
  const AccumArgs* adesc;   // [rounds][n_members], boxes at tile height qtile_rows(m, rb)
  const int* gpre;          // [n_groups + 1]
  const int* wait;          // [n_groups]
  int n_groups, n_members, total;
  int* done;                // [2 n_members][QSLOTS] slots, QSLOT_STRIDE ints apart
  int* head;                // next item
  int* abort;               // set by a wait longer than wait_ticks (s_memrealtime ticks); stops the queue
  long long wait_ticks;
};
// Tile height whose 32-wide tiles take all m * rb threads of the plan (0: the
// plan has fewer than 64 threads and no work-queue launch).
int qtile_rows(int m, int rb);
// grid: the plan's resident workgroups on n_cu compute units (at most total)
hipError_t launch_queue(int m, int rb, const QueueArgs& q, int n_cu, hipStream_t s);
hipError_t clear_i32(int* p, int n, hipStream_t s);
// Level constants, the plan's probe table and the probe spectrum (qspec; spec_tmp:
// m*m + m double2 of scratch).
hipError_t launch_level_constants(int m, int levels, double alpha, int u_given,
                                  const double2* q64, double* u0, double* w0, float* w0f, float* u0f,
                                  float2* qf, double* lvl, int lvl_a_off, double2* scr_q, double* scr_u, int rb,
                                  float4* qtab, float2* qspec, double2* spec_tmp, hipStream_t s);
hipError_t launch_permute_sqrt(int m, int rb, int n_pos, const float* src, int is_sqrt, float* dst,
                               int* bad_flag, hipStream_t s);
hipError_t launch_unpermute_sqrt(int m, int rb, int n_pos, const float* src, float* dst, hipStream_t s);
hipError_t launch_reduce_sum(const double* x, int n, double* out, hipStream_t s);
// per position: sum of nw partials (optionally sqrt), then a fixed-order total
hipError_t launch_reduce_parts(const double* parts, int n, int nw, int take_sqrt, double* per_pos,
                               double* total, hipStream_t s);
hipError_t launch_set_counter(int* counter, int value, hipStream_t s);
hipError_t launch_advance_counter(int* counter, hipStream_t s);
// Q += sum_s num_s / (sum_s den_s + beta sum_s max_s) where the denominator is
// positive; q64 is the FP64 master probe.  Two passes: FP64 sums over fixed
// chunks of PROBE_CHUNK slots (in slot order) into `scratch`, then the chunks in
// order, so the result does not depend on the launch shape.
constexpr int PROBE_CHUNK = 16;
inline size_t probe_scratch_doubles(int m, int max_count) {
  const size_t chunks = (size_t)(max_count + PROBE_CHUNK - 1) / PROBE_CHUNK;
  return chunks * ((size_t)3 * m * m + 1);
}
hipError_t launch_probe_apply(int m, int count, int nwaves, const float2* num, const float* den,
                              const float* pmax, double beta, double2* q64, double* scratch, hipStream_t s);
hipError_t launch_convert_c64_c128(const float2* src, double2* dst, size_t n, hipStream_t s);
hipError_t launch_convert_c128_c64(const double2* src, float2* dst, size_t n, hipStream_t s);
hipError_t launch_check_finite_c64(const float2* src, size_t n, int* bad_flag, hipStream_t s);
hipError_t launch_fill_c64(float2* dst, size_t n, float re, float im, hipStream_t s);

}  // namespace mg
