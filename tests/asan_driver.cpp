// Host AddressSanitizer run of the C ABI: built with the runtime's host code
// instrumented (hipcc -Xarch_host -fsanitize=address; device code is not), it
// goes through every entry point once, with several flag combinations and the
// error paths, on a small reconstruction.  Exit status 0 when every call
// returned what it should; a memory error aborts the run with ASan's report.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "magpie.h"
#include "magpie_learned.h"

namespace {

int failures = 0;

void expect(int got, int want, const char* what) {
  if (got != want) {
    std::fprintf(stderr, "%s: returned %d, expected %d (%s)\n", what, got, want, magpie_last_error());
    ++failures;
  }
}

using c64 = std::complex<float>;

// a disc probe with a quadratic phase, as the synthetic workloads use
std::vector<c64> probe(int m) {
  std::vector<c64> q((size_t)m * m);
  const double R = 10.0 * m / 32.0, c0 = (m - 1) / 2.0;
  for (int y = 0; y < m; ++y)
    for (int x = 0; x < m; ++x) {
      const double r = std::hypot(y - c0, x - c0);
      const double a = r <= R ? 1.0 : std::exp(-(r - R) * (r - R) / (2.0 * (m / 16.0) * (m / 16.0)));
      const double ph = M_PI * r * r / (R * R);
      q[(size_t)y * m + x] = c64((float)(a * std::cos(ph)), (float)(a * std::sin(ph)));
    }
  return q;
}

std::vector<c64> object(int n, int seed) {
  std::vector<c64> z((size_t)n * n);
  for (int y = 0; y < n; ++y)
    for (int x = 0; x < n; ++x) {
      const double ph = 0.8 * std::sin(0.11 * x + 0.07 * y + seed) + 0.3 * std::cos(0.05 * x * y / n);
      const double a = 0.9 + 0.1 * std::cos(0.13 * x - 0.17 * y);
      z[(size_t)y * n + x] = c64((float)(a * std::cos(ph)), (float)(a * std::sin(ph)));
    }
  return z;
}

std::vector<int32_t> raster(int n, int m, int step) {
  std::vector<int32_t> o;
  for (int r = 0; r + m <= n; r += step)
    for (int c = 0; c + m <= n; c += step) {
      o.push_back(r);
      o.push_back(c);
    }
  return o;
}

// one context with data from the library's own forward model of `truth`
magpie_ctx* context(int n, int m, int L, const std::vector<c64>& truth, std::vector<int32_t>& offs) {
  magpie_ctx* c = nullptr;
  expect(magpie_create(&c, n, n, m, L, 0.5, 0, nullptr), MAGPIE_OK, "create");
  const auto q = probe(m);
  expect(magpie_set_probe(c, q.data(), MAGPIE_C64, 0), MAGPIE_OK, "set_probe");
  offs = raster(n, m, m / 4);
  expect(magpie_set_positions(c, (int)(offs.size() / 2), offs.data()), MAGPIE_OK, "set_positions");
  std::vector<float> d((offs.size() / 2) * m * m);
  expect(magpie_forward_model(c, truth.data(), 0, d.data(), 0), MAGPIE_OK, "forward_model");
  expect(magpie_load_intensities(c, d.data(), 0, 0), MAGPIE_OK, "load_intensities");
  return c;
}

}  // namespace

int main() {
  const int n = 96, m = 16;
  const auto truth = object(n, 1);
  std::vector<int32_t> offs;
  magpie_ctx* c = context(n, m, 3, truth, offs);
  const int N = (int)(offs.size() / 2);

  // plain epochs, objective, outputs, timing, tuning
  std::vector<c64> ones((size_t)n * n, c64(1.0f, 0.0f)), z((size_t)n * n), qo((size_t)m * m);
  expect(magpie_set_object(c, ones.data(), MAGPIE_C64, 0), MAGPIE_OK, "set_object");
  expect(magpie_run_epochs(c, 2, 7, 11, nullptr), MAGPIE_OK, "run_epochs");
  double phi = 0, stat = 0;
  expect(magpie_objective(c, &phi, &stat), MAGPIE_OK, "objective");
  std::vector<double> phik(N);
  expect(magpie_get_step_phi(c, phik.data()), MAGPIE_OK, "get_step_phi");
  expect(magpie_get_object(c, z.data(), MAGPIE_C64, 0), MAGPIE_OK, "get_object");
  std::vector<std::complex<double>> z128((size_t)n * n);
  expect(magpie_get_object(c, z128.data(), MAGPIE_C128, 0), MAGPIE_OK, "get_object c128");
  expect(magpie_get_probe(c, qo.data(), MAGPIE_C64, 0), MAGPIE_OK, "get_probe");
  expect(magpie_set_timing(c, 1), MAGPIE_OK, "set_timing");
  expect(magpie_run_epochs(c, 1, 16, 11, nullptr), MAGPIE_OK, "run_epochs timed");
  double sms = 0, ams = 0;
  int64_t sl = 0, al = 0, np = 0;
  expect(magpie_get_timing(c, &sms, &ams, &sl, &al, &np), MAGPIE_OK, "get_timing");
  expect(magpie_set_timing(c, 0), MAGPIE_OK, "set_timing off");
  int32_t plans[8];
  const int np_ = magpie_list_plans(m, plans, 8);
  if (np_ < 1) ++failures;
  for (int i = 0; i < np_; ++i) expect(magpie_set_tuning(c, plans[i], 8 << (i % 3)), MAGPIE_OK, "set_tuning");
  double su = 0, au = 0;
  expect(magpie_autotune(c, 7, 1, &su, &au), MAGPIE_OK, "autotune");
  int rb = 0, th = 0;
  expect(magpie_get_tuning(c, &rb, &th), MAGPIE_OK, "get_tuning");
  uint64_t ep = 0;
  expect(magpie_get_epoch_index(c, &ep), MAGPIE_OK, "get_epoch_index");
  expect(magpie_set_epoch_index(c, ep + 3), MAGPIE_OK, "set_epoch_index");
  std::vector<int32_t> order(N);
  expect(magpie_permutation(5, 0, N, order.data()), MAGPIE_OK, "permutation");
  expect(magpie_run_epochs(c, 1, N, 0, order.data()), MAGPIE_OK, "run_epochs order");
  expect(magpie_run_epochs_noalloc(c, 2, 7, 11), MAGPIE_OK, "run_epochs_noalloc");
  expect(magpie_run_minibatch(c, std::min(N, 5), order.data()), MAGPIE_OK, "run_minibatch");
  expect(magpie_run_minibatch(c, N, order.data()), MAGPIE_OK, "run_minibatch all");
  {
    std::vector<int32_t> twice = {order[0], order[0]};
    expect(magpie_run_minibatch(c, 2, twice.data()), MAGPIE_ERR_INVALID_ARG, "run_minibatch repeated");
    expect(magpie_run_minibatch(c, N + 1, order.data()), MAGPIE_ERR_INVALID_ARG, "run_minibatch too many");
  }
  std::vector<double> u((size_t)m * m, 0.1);
  expect(magpie_set_regularization(c, 0.0, u.data()), MAGPIE_OK, "set_regularization u");
  expect(magpie_set_regularization(c, 0.5, nullptr), MAGPIE_OK, "set_regularization alpha");

  // every flag, with graphs, buffers growing between calls
  const uint32_t all = MAGPIE_UPDATE_PROBE | MAGPIE_PROBE_ALTERNATE | MAGPIE_PHASE_RECYCLE | MAGPIE_GRAPH;
  expect(magpie_set_flags(c, all, 0.3), MAGPIE_OK, "set_flags all");
  expect(magpie_run_epochs(c, 2, 5, 3, nullptr), MAGPIE_OK, "run_epochs all flags");
  expect(magpie_run_epochs(c, 3, 40, 3, nullptr), MAGPIE_OK, "run_epochs larger batch");
  expect(magpie_set_flags(c, MAGPIE_UPDATE_PROBE, 0.3), MAGPIE_OK, "set_flags probe");
  expect(magpie_run_epochs_noalloc(c, 1, 5, 3), MAGPIE_ERR_UNSUPPORTED, "run_epochs_noalloc with probe step");
  expect(magpie_run_epochs(c, 1, 5, 3, nullptr), MAGPIE_OK, "run_epochs probe");
  expect(magpie_set_flags(c, 0, 0.0), MAGPIE_OK, "set_flags none");
  expect(magpie_sync(c), MAGPIE_OK, "sync");

  // error paths
  expect(magpie_set_flags(c, MAGPIE_PROBE_ALTERNATE, 0.0), MAGPIE_ERR_INVALID_ARG, "alternate alone");
  expect(magpie_set_flags(c, 0x100u, 0.0), MAGPIE_ERR_INVALID_ARG, "unknown flag");
  expect(magpie_run_epochs(c, 1, 0, 0, nullptr), MAGPIE_ERR_INVALID_ARG, "batch 0");
  std::vector<int32_t> bad = {0, 0, n, 0};
  expect(magpie_set_positions(c, 2, bad.data()), MAGPIE_ERR_INVALID_ARG, "offset out of range");
  std::vector<int32_t> notperm(N, 0);
  expect(magpie_run_epochs(c, 1, 4, 0, notperm.data()), MAGPIE_ERR_INVALID_ARG, "order not a permutation");
  expect(magpie_set_tuning(c, 3, 0), MAGPIE_ERR_UNSUPPORTED, "no such plan");
  expect(magpie_set_tuning(c, 0, 4), MAGPIE_ERR_UNSUPPORTED, "no such tile height");
  magpie_ctx* e = nullptr;
  expect(magpie_create(&e, 64, 64, 24, 2, 0.5, 0, nullptr), MAGPIE_ERR_UNSUPPORTED, "m not a power of two");
  expect(magpie_create(&e, 64, 64, 16, 2, 0.5, 0, nullptr), MAGPIE_OK, "create fresh");
  expect(magpie_run_epochs(e, 1, 4, 0, nullptr), MAGPIE_ERR_BAD_STATE, "run before data");
  expect(magpie_objective(e, &phi, nullptr), MAGPIE_ERR_BAD_STATE, "objective before data");
  expect(magpie_destroy(e), MAGPIE_OK, "destroy fresh");
  expect(magpie_destroy(nullptr), MAGPIE_OK, "destroy NULL");
  std::vector<float> dneg((size_t)N * m * m, -1.0f);
  expect(magpie_load_intensities(c, dneg.data(), 0, 0), MAGPIE_ERR_NUMERIC, "negative intensities");

  // two contexts in one multi-reconstruction run (the second a different size)
  std::vector<int32_t> offs2;
  const auto truth2 = object(64, 2);
  magpie_ctx* c2 = context(64, m, 2, truth2, offs2);
  magpie_ctx* c1 = context(n, m, 3, truth, offs);
  magpie_ctx* both[2] = {c1, c2};
  const int batches[2] = {9, 5};
  expect(magpie_run_epochs_multi(both, 2, 2, batches, 7), MAGPIE_OK, "run_epochs_multi");
  expect(magpie_set_flags(c2, MAGPIE_PHASE_RECYCLE, 0.0), MAGPIE_OK, "set_flags c2");
  expect(magpie_run_epochs_multi(both, 2, 1, batches, 7), MAGPIE_ERR_UNSUPPORTED, "multi with recycling");
  // the work-queue launch: mixed flags refused, then both contexts over 10 epochs (chunks
  // 1 + 8 + 1), then one context alone through run_epochs
  expect(magpie_set_flags(c2, MAGPIE_PERSISTENT, 0.0), MAGPIE_OK, "set_flags c2 persistent");
  expect(magpie_run_epochs_multi(both, 2, 1, batches, 7), MAGPIE_ERR_INVALID_ARG, "multi with mixed persistent");
  expect(magpie_set_flags(c1, MAGPIE_PERSISTENT, 0.0), MAGPIE_OK, "set_flags c1 persistent");
  expect(magpie_run_epochs_multi(both, 2, 10, batches, 7), MAGPIE_OK, "run_epochs_multi queue");
  expect(magpie_run_epochs(c2, 2, 5, 3, nullptr), MAGPIE_OK, "run_epochs queue");
  expect(magpie_run_epochs(c2, 1, 5, 3, notperm.data()), MAGPIE_ERR_UNSUPPORTED, "queue with caller orders");

  // the 64-point plans (512- and 256-thread workgroups) with graphs and every flag
  {
    const int n64 = 160, m64 = 64;
    const auto t64 = object(n64, 3);
    std::vector<int32_t> o64;
    magpie_ctx* ctx64 = context(n64, m64, 3, t64, o64);
    std::vector<c64> one64((size_t)n64 * n64, c64(1.0f, 0.0f)), z64((size_t)n64 * n64);
    expect(magpie_set_object(ctx64, one64.data(), MAGPIE_C64, 0), MAGPIE_OK, "set_object m64");
    expect(magpie_run_epochs(ctx64, 2, 13, 1, nullptr), MAGPIE_OK, "run_epochs m64");
    expect(magpie_set_flags(ctx64, all, 0.3), MAGPIE_OK, "set_flags m64");
    expect(magpie_run_epochs(ctx64, 2, 13, 1, nullptr), MAGPIE_OK, "run_epochs m64 all flags");
    expect(magpie_run_epochs(ctx64, 1, 49, 1, nullptr), MAGPIE_OK, "run_epochs m64 one minibatch");
    expect(magpie_set_flags(ctx64, MAGPIE_GRAPH | MAGPIE_PHASE_RECYCLE, 0.0), MAGPIE_OK, "set_flags m64 graph");
    expect(magpie_autotune(ctx64, 13, 1, &su, &au), MAGPIE_OK, "autotune m64");
    const int32_t cands[3] = {5, 13, 1000};
    int32_t bb = 0;
    double rr[3] = {0.0, 0.0, 0.0};
    expect(magpie_autotune_batch(ctx64, cands, 3, 1, &bb, rr), MAGPIE_OK, "autotune_batch m64");
    expect(magpie_autotune_batch(ctx64, cands, 0, 1, &bb, rr), MAGPIE_ERR_INVALID_ARG, "autotune_batch none");
    expect(magpie_autotune_batch(ctx64, cands, 3, 1, nullptr, rr), MAGPIE_ERR_INVALID_ARG, "autotune_batch NULL");
    expect(magpie_set_tuning(ctx64, 4, 16), MAGPIE_OK, "set_tuning m64");
    expect(magpie_run_epochs(ctx64, 3, 13, 1, nullptr), MAGPIE_OK, "run_epochs m64 plan 4");
    expect(magpie_set_flags(ctx64, MAGPIE_PERSISTENT, 0.0), MAGPIE_OK, "set_flags m64 persistent");
    expect(magpie_run_epochs(ctx64, 2, 13, 1, nullptr), MAGPIE_OK, "run_epochs m64 plan 4 queue");
    expect(magpie_objective(ctx64, &phi, &stat), MAGPIE_OK, "objective m64");
    expect(magpie_get_object(ctx64, z64.data(), MAGPIE_C64, 0), MAGPIE_OK, "get_object m64");
    expect(magpie_destroy(ctx64), MAGPIE_OK, "destroy m64");
  }

  // learned start: network, loss, training step, input map, pyramid
  magpie_cnn* net = nullptr;
  const int side = 8;
  expect(magpie_cnn_create(&net, 3, 32, side, 2, MAGPIE_W_F32, 0, nullptr), MAGPIE_OK, "cnn_create");
  int64_t np2 = 0;
  expect(magpie_cnn_num_params(net, &np2), MAGPIE_OK, "cnn_num_params");
  std::vector<float> params((size_t)np2);
  for (size_t i = 0; i < params.size(); ++i) params[i] = 0.01f * (float)std::sin(0.37 * (double)i);
  expect(magpie_cnn_set_params(net, params.data(), 0), MAGPIE_OK, "cnn_set_params");
  std::vector<float> x((size_t)2 * 3 * side * side, 0.5f), y((size_t)2 * 2 * (2 * side) * (2 * side));
  expect(magpie_cnn_forward(net, x.data(), y.data(), 2, 0), MAGPIE_OK, "cnn_forward");
  std::vector<c64> target((size_t)2 * (2 * side) * (2 * side), c64(1.0f, 0.1f));
  std::vector<float> mask((size_t)(2 * side) * (2 * side), 1.0f);
  double loss = 0;
  expect(magpie_cnn_loss(net, target.data(), mask.data(), 2, 1, 0, &loss), MAGPIE_OK, "cnn_loss");
  expect(magpie_cnn_backward(net, nullptr, 2, 0), MAGPIE_OK, "cnn_backward");
  std::vector<float> grads((size_t)np2);
  expect(magpie_cnn_get_grads(net, grads.data(), 0), MAGPIE_OK, "cnn_get_grads");
  expect(magpie_cnn_adam_step(net, 1e-3f, 0.9f, 0.999f, 1e-8f), MAGPIE_OK, "cnn_adam_step");
  expect(magpie_cnn_get_params(net, params.data(), 0), MAGPIE_OK, "cnn_get_params");
  expect(magpie_cnn_sync(net), MAGPIE_OK, "cnn_sync");
  std::vector<float> map((size_t)4 * 16 * 16);
  expect(magpie_input_map(c1, 16, map.data(), 0), MAGPIE_OK, "input_map");
  std::vector<c64> coarse((size_t)(n / 4) * (n / 4), c64(1.0f, 0.0f));
  expect(magpie_set_object_from_coarse(c1, coarse.data(), n / 4, MAGPIE_COARSE_C64, 0), MAGPIE_OK,
         "set_object_from_coarse");
  magpie_cnn* net16 = nullptr;
  expect(magpie_cnn_create(&net16, 4, 32, 12, 1, MAGPIE_W_BF16, 0, nullptr), MAGPIE_OK, "cnn_create bf16");
  double pl = 0, pf = 0;
  int used = 0;
  expect(magpie_learned_start(c1, net16, &pl, &pf, &used), MAGPIE_OK, "learned_start");
  expect(magpie_cnn_forward(net, x.data(), y.data(), 3, 0), MAGPIE_ERR_INVALID_ARG, "cnn batch too large");
  expect(magpie_cnn_destroy(net16), MAGPIE_OK, "cnn_destroy bf16");
  expect(magpie_cnn_destroy(net), MAGPIE_OK, "cnn_destroy");

  expect(magpie_destroy(c1), MAGPIE_OK, "destroy c1");
  expect(magpie_destroy(c2), MAGPIE_OK, "destroy c2");
  expect(magpie_destroy(c), MAGPIE_OK, "destroy");
  std::printf("asan driver: %d unexpected return codes\n", failures);
  std::fflush(stdout);
  // Leave without running the HIP and HSA runtimes' static destructors: under
  // ASan their teardown can free memory through the sanitizer's device-memory
  // allocator after that allocator is unloaded (a CHECK failure inside the
  // runtimes, outside this library).  Every context was destroyed above.
  std::_Exit(failures == 0 ? 0 : 1);
}
