// magpie_run_epochs_noalloc: the epochs of magpie_run_epochs (seeded library
// permutations) with every per-call buffer taken from a fixed file-scope device
// array instead of device allocations, for callers that cannot allocate.
//
// The array holds, from its start: the minibatch staging [B][m][m] float2 (the
// c_k = w0 dz_k the step kernel writes and the accumulation reads), then for a
// chunk of epochs the position records (k, row, col, 0) [E][N] in processing
// order and the inverse permutations [E][N].  Each chunk's permutations are drawn
// on the device by the same splitmix64 Fisher-Yates as the host's
// (magpie_permutation), so the results equal magpie_run_epochs bit for bit.
// Every value is written before it is read within a call, so nothing needs
// clearing; calls on one device share the array (it keeps the last call's
// contents), and calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "context.h"

using namespace mgrt;

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)16 << 20;   // per device, held until the process ends
constexpr int MAX_DEVICES = 64;
constexpr int MAX_POSITIONS = 16384;                  // permutation and its draws in LDS: 8 N bytes
constexpr int PERM_THREADS = 256;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
unsigned char* g_scratch[MAX_DEVICES] = {};

// One workgroup per epoch e of the chunk: the Fisher-Yates shuffle of 0..n-1 with
// j_i = next() mod (i + 1) for i = n-1 .. 1, where next() are the outputs of
// splitmix64 from state seed XOR (epoch0 + e).  Output t of splitmix64 is the
// finaliser of state + (t + 1) * 0x9E3779B97F4A7C15 (the state only advances by
// that constant), so every thread draws its share of the j_i at once; one thread
// then performs the swaps in LDS.  Records (k, row, col, 0) and the inverse
// permutation follow in parallel.
__global__ __launch_bounds__(PERM_THREADS) void permutation_records_kernel(uint64_t seed, uint64_t epoch0, int n,
                                                                         const int2* __restrict__ offs,
                                                                         int4* __restrict__ posrec,
                                                                         int* __restrict__ inv) {
  extern __shared__ int lds_perm[];
  int* perm = lds_perm;
  int* draw = lds_perm + n;
  const int e = (int)blockIdx.x;
  const uint64_t s0 = seed ^ (epoch0 + (uint64_t)e);
  for (int i = threadIdx.x; i < n; i += PERM_THREADS) {
    perm[i] = i;
    if (i > 0) {
      const uint64_t t = (uint64_t)(n - 1 - i);   // i = n-1 takes the first output
      uint64_t z = s0 + (t + 1) * 0x9E3779B97F4A7C15ull;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      draw[i] = (int)(z % (uint64_t)(i + 1));
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = n - 1; i > 0; --i) {
      const int j = draw[i];
      const int a = perm[i];
      perm[i] = perm[j];
      perm[j] = a;
    }
  }
  __syncthreads();
  int4* rec = posrec + (size_t)e * n;
  int* iv = inv + (size_t)e * n;
  for (int i = threadIdx.x; i < n; i += PERM_THREADS) {
    const int k = perm[i];
    const int2 o = offs[k];
    rec[i] = make_int4(k, o.x, o.y, 0);
    iv[k] = i;
  }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// Resolves the device address of this device's scratch array (once per device,
// with that device current); called when a context is created on it.
int mgrt::noalloc_init_device(int device) {
  if (device < 0 || device >= MAX_DEVICES) return fail(MAGPIE_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return MAGPIE_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(MAGPIE_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch[device] = static_cast<unsigned char*>(p);
  return MAGPIE_OK;
}

extern "C" int magpie_run_epochs_noalloc(magpie_ctx* c, int n_epochs, int batch, uint64_t seed) {
  if (!c) return fail(MAGPIE_ERR_INVALID_ARG, "NULL context");
  if (!c->has_probe || !c->has_pos || !c->has_data)
    return fail(MAGPIE_ERR_BAD_STATE, "set probe, positions and intensities first");
  if (n_epochs < 0 || batch < 1) return fail(MAGPIE_ERR_INVALID_ARG, "n_epochs >= 0 and batch >= 1 required");
  if (n_epochs == 0) return MAGPIE_OK;
  if (c->flags & MAGPIE_UPDATE_PROBE)
    return fail(MAGPIE_ERR_UNSUPPORTED, "the probe step needs buffers this entry point does not hold; "
                                        "use magpie_run_epochs");
  const int N = c->n_pos, m = c->m;
  const int B = std::min(batch, N);
  if (N > MAX_POSITIONS)
    return fail(MAGPIE_ERR_UNSUPPORTED, "more than 16384 positions (the on-device permutation's limit)");
  const size_t stage_bytes = align256((size_t)B * m * m * sizeof(float2));
  const size_t epoch_bytes = (size_t)N * (sizeof(int4) + sizeof(int));
  if (stage_bytes + epoch_bytes > SCRATCH_BYTES)
    return fail(MAGPIE_ERR_UNSUPPORTED,
                "minibatch staging (8 B m^2 per position) plus one epoch's records (20 B per position) exceed "
                "the 16 MiB scratch: use a smaller minibatch or magpie_run_epochs");
  int rc = set_dev(c);
  if (rc) return rc;
  unsigned char* base = (c->device >= 0 && c->device < MAX_DEVICES) ? g_scratch[c->device] : nullptr;
  if (!base) return fail(MAGPIE_ERR_BAD_STATE, "scratch of this device not resolved");
  const int e_chunk = (int)std::min<size_t>((size_t)n_epochs, (SCRATCH_BYTES - stage_bytes) / epoch_bytes);
  float2* stage = reinterpret_cast<float2*>(base);
  int4* posrec = reinterpret_cast<int4*>(base + stage_bytes);
  int* inv = reinterpret_cast<int*>(base + stage_bytes + (size_t)e_chunk * N * sizeof(int4));
  const size_t lds = (size_t)2 * N * sizeof(int);
  MG_HIP(hipFuncSetAttribute((const void*)permutation_records_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds));
  const bool timing = c->timing;   // per-launch events are created on demand: not here
  c->timing = false;
  for (int e0 = 0; e0 < n_epochs && rc == MAGPIE_OK; e0 += e_chunk) {
    const int ne = std::min(e_chunk, n_epochs - e0);
    hipLaunchKernelGGL(permutation_records_kernel, dim3(ne), dim3(PERM_THREADS), lds, c->stream, seed,
                       c->epoch_index + (uint64_t)e0, N, (const int2*)c->offs, posrec, inv);
    const hipError_t le = hipGetLastError();
    if (le != hipSuccess) {
      rc = fail(MAGPIE_ERR_HIP, std::string("permutation kernel: ") + hipGetErrorString(le));
      break;
    }
    rc = launch_epochs(c, ne, B, (N + B - 1) / B, false, EpochBuffers{stage, posrec, inv, nullptr});
  }
  c->timing = timing;
  if (rc) return rc;
  c->epoch_index += (uint64_t)n_epochs;
  return MAGPIE_OK;
}
