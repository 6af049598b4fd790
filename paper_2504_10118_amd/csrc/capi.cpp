// Host runtime of the MAGPIE C ABI (include/magpie.h): context, device
// buffers, input validation, epoch scheduling and kernel launches.
#include <chrono>
#include <mutex>

#include "context.h"

using namespace mgrt;

namespace {

void drop_graph(magpie_ctx* c) {
  if (c->gexec) hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
  c->g_batch = 0;
}

// eq. (3.2) phase store: sized for the current positions and reset to theta = 0
// (factor 1) while MAGPIE_PHASE_RECYCLE is on, freed while it is off.
int reset_phases(magpie_ctx* c) {
  const bool on = (c->flags & MAGPIE_PHASE_RECYCLE) && c->has_pos;
  const size_t need = on ? (size_t)c->n_pos * c->m * c->m : 0;
  if (!on || need != c->phase_cap) {
    drop_graph(c);
    dev_free(c->phase);
    c->phase_cap = 0;
  }
  if (!on) return MAGPIE_OK;
  if (!c->phase) {
    int rc = dev_alloc(&c->phase, need);
    if (rc) return rc;
    c->phase_cap = need;
  }
  MG_HIP(mg::launch_fill_c64(c->phase, need, 1.0f, 0.0f, c->stream));
  return MAGPIE_OK;
}

int free_positions(magpie_ctx* c) {
  drop_graph(c);
  dev_free(c->phase);
  c->phase_cap = 0;
  dev_free(c->offs);
  dev_free(c->sqrtd);
  dev_free(c->phi_step);
  dev_free(c->phi_obj);
  dev_free(c->gnorm);
  dev_free(c->step_part);
  dev_free(c->obj_part);
  dev_free(c->gn_part);
  dev_free(c->tile_ptr);
  dev_free(c->tile_ent);
  c->has_pos = false;
  c->has_data = false;
  c->n_pos = 0;
  return MAGPIE_OK;
}

int rebuild_levels(magpie_ctx* c) {
  MG_HIP(mg::launch_level_constants(c->m, c->L, c->alpha, c->u_given ? 1 : 0, c->q64, c->u0, c->w0, c->w0f, c->u0f,
                                    c->qf, c->lvl, c->lvl_a_off, c->scr_q, c->scr_u, c->rb, c->qtab, c->qspec,
                                    c->spec_tmp, c->stream));
  return MAGPIE_OK;
}

hipEvent_t take_event(magpie_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Events for a timed launch (recorded by the dispatch itself at kernel start
// and end); returns the index into c->timed or -1 when timing is off.
int timed_slot(magpie_ctx* c, int kind, int count) {
  if (!c->timing) return -1;
  magpie_ctx::Timed t{take_event(c), take_event(c), kind, count};
  if (!t.a || !t.b) {   // untimed launch; an event already taken goes back to the pool
    if (t.a) c->ev_pool.push_back(t.a);
    if (t.b) c->ev_pool.push_back(t.b);
    return -1;
  }
  c->timed.push_back(t);
  return (int)c->timed.size() - 1;
}

// The library's own streams of a device (default priority, non-blocking), created
// on first use and kept until the process ends: multi-context runs put all but
// the first partition of their reconstructions on them.
int side_stream(int device, int index, hipStream_t* out) {
  static std::mutex mu;
  static std::vector<std::vector<hipStream_t>> pool;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)pool.size() <= device) pool.resize((size_t)device + 1);
  auto& v = pool[(size_t)device];
  while ((int)v.size() <= index) {
    hipStream_t sN = nullptr;
    MG_HIP(hipStreamCreateWithFlags(&sN, hipStreamNonBlocking));
    v.push_back(sN);
  }
  *out = v[(size_t)index];
  return MAGPIE_OK;
}

// Round descriptors of a multi-context chunk: pinned host and device slot `slot`
// of the first context, grown to `bytes`, once its previous upload is done.
int multi_slot(magpie_ctx* c, int slot, size_t bytes) {
  if (c->mdesc_pending[slot]) {
    MG_HIP(hipEventSynchronize(c->mdesc_done[slot]));
    c->mdesc_pending[slot] = false;
  }
  if (bytes <= c->mdesc_cap[slot]) return MAGPIE_OK;
  if (c->mdesc_host[slot]) hipHostFree(c->mdesc_host[slot]);
  c->mdesc_host[slot] = nullptr;
  dev_free(c->mdesc_dev[slot]);
  c->mdesc_cap[slot] = 0;
  const size_t cap = std::max(bytes, (size_t)1 << 20);
  if (hipHostMalloc(&c->mdesc_host[slot], cap, hipHostMallocDefault) != hipSuccess) {
    c->mdesc_host[slot] = nullptr;
    return fail(MAGPIE_ERR_OOM, "pinned host allocation failed");
  }
  unsigned char* d = nullptr;
  int rc = dev_alloc(&d, cap);
  if (rc) return rc;
  c->mdesc_dev[slot] = d;
  c->mdesc_cap[slot] = cap;
  return MAGPIE_OK;
}

// Per-tile ascending lists of overlapping positions (with their offsets) for
// the context's tile height.
int build_tiles(magpie_ctx* c) {
  const int m = c->m, n_pos = c->n_pos;
  const int32_t* offsets = c->h_offs.data();
  dev_free(c->tile_ptr);
  dev_free(c->tile_ent);
  c->tiles_x = (c->nc + mg::ACC_TILE_W - 1) / mg::ACC_TILE_W;
  c->tiles_y = (c->nr + c->th - 1) / c->th;
  const int nt = c->tiles_x * c->tiles_y;
  // the box of tiles some window reaches (the accumulation runs over it only)
  int r0 = c->nr, r1 = 0, c0 = c->nc, c1 = 0;
  for (int k = 0; k < n_pos; ++k) {
    r0 = std::min(r0, offsets[2 * k]);
    r1 = std::max(r1, offsets[2 * k] + m - 1);
    c0 = std::min(c0, offsets[2 * k + 1]);
    c1 = std::max(c1, offsets[2 * k + 1] + m - 1);
  }
  c->scan_r0 = r0;
  c->scan_r1 = r1;
  c->box_x0 = c0 / mg::ACC_TILE_W;
  c->box_y0 = r0 / c->th;
  c->box_nx = c1 / mg::ACC_TILE_W - c->box_x0 + 1;
  c->box_ny = r1 / c->th - c->box_y0 + 1;
  std::vector<std::vector<int>> lists(nt);
  for (int k = 0; k < n_pos; ++k) {
    const int r = offsets[2 * k], cc = offsets[2 * k + 1];
    for (int ty = r / c->th; ty <= (r + m - 1) / c->th; ++ty)
      for (int tx = cc / mg::ACC_TILE_W; tx <= (cc + m - 1) / mg::ACC_TILE_W; ++tx)
        lists[ty * c->tiles_x + tx].push_back(k);
  }
  std::vector<int> ptr(nt + 1, 0);
  std::vector<int4> pos;
  for (int t = 0; t < nt; ++t) {
    ptr[t + 1] = ptr[t] + (int)lists[t].size();
    for (int k : lists[t]) pos.push_back(make_int4(k, offsets[2 * k], offsets[2 * k + 1], 0));
  }
  int rc = dev_alloc(&c->tile_ptr, nt + 1);
  if (!rc) rc = dev_alloc(&c->tile_ent, std::max<size_t>(pos.size(), 1));
  if (rc) return rc;
  MG_HIP(hipMemcpyAsync(c->tile_ptr, ptr.data(), ptr.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
  if (!pos.empty())
    MG_HIP(hipMemcpyAsync(c->tile_ent, pos.data(), pos.size() * sizeof(int4), hipMemcpyHostToDevice, c->stream));
  MG_HIP(hipStreamSynchronize(c->stream));
  drop_graph(c);
  return MAGPIE_OK;
}

}  // namespace

extern "C" {

const char* magpie_last_error(void) { return g_last_error.c_str(); }

int magpie_create(magpie_ctx** out, int n_rows, int n_cols, int m, int n_levels, double alpha, int device,
                  void* hip_stream) {
  if (!out) return fail(MAGPIE_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!valid_m(m)) return fail(MAGPIE_ERR_UNSUPPORTED, "m must be one of 8, 16, 32, 64, 128");
  if (n_levels < 1 || n_levels > ilog2(m) + 1)
    return fail(MAGPIE_ERR_UNSUPPORTED, "n_levels must be in [1, log2(m)+1]");
  if (n_rows < m || n_cols < m) return fail(MAGPIE_ERR_INVALID_ARG, "object smaller than the probe");
  // the kernels address the object through 32-bit buffer ranges
  if ((uint64_t)n_rows * (uint64_t)n_cols * sizeof(float2) >= (1ull << 32))
    return fail(MAGPIE_ERR_UNSUPPORTED, "object of 2^32 bytes or more (n_rows * n_cols >= 2^29)");
  if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(MAGPIE_ERR_INVALID_ARG, "alpha must be finite, >= 0");
  int ndev = 0;
  MG_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(MAGPIE_ERR_INVALID_ARG, "no such device");

  magpie_ctx* c = new magpie_ctx();
  c->device = device;
  c->nr = n_rows;
  c->nc = n_cols;
  c->m = m;
  c->L = n_levels;
  c->alpha = alpha;
  c->rb = mg::default_plan(m);
  int rc = set_dev(c);
  if (!rc) rc = noalloc_init_device(device);
  if (rc) { delete c; return rc; }
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->n_cu < 1)
    c->n_cu = 256;
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(MAGPIE_ERR_HIP, "hipStreamCreate failed");
    }
    c->own_stream = true;
  }
  const size_t mm = (size_t)m * m;
  const size_t half = (size_t)(m / 2) * (m / 2);
  size_t nlvl = 0;
  for (int l = 1; l < n_levels; ++l) nlvl += 3 * (size_t)(m >> l) * (m >> l);
  nlvl = (nlvl + 1) & ~(size_t)1;          // the A block starts 16-byte aligned (read as double pairs)
  c->lvl_a_off = (int)nlvl;
  nlvl += (size_t)mg::cst_count(m, n_levels);  // the in-wave V-cycle block: A_l per level-1 bin, copies of V_l
  nlvl += 2;                               // a pair read may cover one double past the block
  rc = dev_alloc(&c->z, (size_t)n_rows * n_cols);
  if (!rc) rc = dev_alloc(&c->qf, mm);
  if (!rc) rc = dev_alloc(&c->qtab, mm);
  if (!rc) rc = dev_alloc(&c->qspec, mm);
  if (!rc) rc = dev_alloc(&c->spec_tmp, mm + (size_t)m);   // row transforms, then row sums of |Q|
  if (!rc) rc = dev_alloc(&c->q64, mm);
  if (!rc) rc = dev_alloc(&c->u0, mm);
  if (!rc) rc = dev_alloc(&c->w0, mm);
  if (!rc) rc = dev_alloc(&c->w0f, mm);
  if (!rc) rc = dev_alloc(&c->u0f, mm);
  if (!rc) rc = dev_alloc(&c->lvl, std::max<size_t>(nlvl, 1));
  if (!rc) rc = dev_alloc(&c->scr_q, 2 * half);
  if (!rc) rc = dev_alloc(&c->scr_u, 2 * half);
  if (!rc) rc = dev_alloc(&c->flag, 1);
  if (!rc) rc = dev_alloc(&c->red, 4);
  if (!rc) rc = dev_alloc(&c->epoch_ctr, 1);
  if (!rc && (hipEventCreateWithFlags(&c->pin_done[0], hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&c->pin_done[1], hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&c->mdesc_done[0], hipEventDisableTiming) != hipSuccess ||
              hipEventCreateWithFlags(&c->mdesc_done[1], hipEventDisableTiming) != hipSuccess))
    rc = fail(MAGPIE_ERR_HIP, "hipEventCreate failed");
  if (rc) {
    magpie_destroy(c);
    return rc;
  }
  // initial object: all ones
  {
    std::vector<float2> ones((size_t)n_rows * n_cols, make_float2(1.0f, 0.0f));
    if (hipMemcpy(c->z, ones.data(), ones.size() * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess) {
      magpie_destroy(c);
      return fail(MAGPIE_ERR_HIP, "object init copy failed");
    }
  }
  if (mg::init_twiddles(c->stream) != hipSuccess) {
    magpie_destroy(c);
    return fail(MAGPIE_ERR_HIP, "twiddle init failed");
  }
  *out = c;
  return MAGPIE_OK;
}

int magpie_destroy(magpie_ctx* c) {
  if (!c) return MAGPIE_OK;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  free_positions(c);
  dev_free(c->z);
  dev_free(c->qf);
  dev_free(c->qtab);
  dev_free(c->qspec);
  dev_free(c->spec_tmp);
  dev_free(c->qctr);
  dev_free(c->q64);
  dev_free(c->u0);
  dev_free(c->w0);
  dev_free(c->w0f);
  dev_free(c->u0f);
  dev_free(c->lvl);
  dev_free(c->scr_q);
  dev_free(c->scr_u);
  dev_free(c->flag);
  dev_free(c->red);
  dev_free(c->epoch_ctr);
  dev_free(c->stage);
  dev_free(c->pnum);
  dev_free(c->pden);
  dev_free(c->pmax);
  dev_free(c->pacc);
  dev_free(c->posrec);
  dev_free(c->posx);
  dev_free(c->inv);
  dev_free(c->lrn_sd);
  dev_free(c->lrn_stats);
  dev_free(c->lrn_fine);
  dev_free(c->lrn_map);
  dev_free(c->lrn_q);
  dev_free(c->lrn_one);
  if (c->h_pin) hipHostFree(c->h_pin);
  for (hipEvent_t ev : c->pin_done)
    if (ev) hipEventDestroy(ev);
  for (int k = 0; k < 2; ++k) {
    if (c->mdesc_done[k]) hipEventDestroy(c->mdesc_done[k]);
    if (c->mdesc_host[k]) hipHostFree(c->mdesc_host[k]);
    dev_free(c->mdesc_dev[k]);
  }
  for (auto& t : c->timed) {
    hipEventDestroy(t.a);
    hipEventDestroy(t.b);
  }
  for (auto e : c->ev_pool) hipEventDestroy(e);
  if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
  delete c;
  return MAGPIE_OK;
}

int magpie_set_probe(magpie_ctx* c, const void* probe, int dtype, int on_device) {
  if (!c || !probe) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  if (dtype != MAGPIE_C64 && dtype != MAGPIE_C128) return fail(MAGPIE_ERR_INVALID_ARG, "bad dtype");
  int rc = set_dev(c);
  if (rc) return rc;
  const size_t mm = (size_t)c->m * c->m;
  std::vector<double2> h(mm);
  if (on_device) {
    if (dtype == MAGPIE_C64) {
      std::vector<float2> t(mm);
      MG_HIP(hipMemcpyAsync(t.data(), probe, mm * sizeof(float2), hipMemcpyDeviceToHost, c->stream));
      MG_HIP(hipStreamSynchronize(c->stream));
      for (size_t i = 0; i < mm; ++i) h[i] = make_double2(t[i].x, t[i].y);
    } else {
      MG_HIP(hipMemcpyAsync(h.data(), probe, mm * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
      MG_HIP(hipStreamSynchronize(c->stream));
    }
  } else if (dtype == MAGPIE_C64) {
    const float2* p = (const float2*)probe;
    for (size_t i = 0; i < mm; ++i) h[i] = make_double2(p[i].x, p[i].y);
  } else {
    std::memcpy(h.data(), probe, mm * sizeof(double2));
  }
  double mx = 0.0;
  for (size_t i = 0; i < mm; ++i) {
    if (!std::isfinite(h[i].x) || !std::isfinite(h[i].y)) return fail(MAGPIE_ERR_NUMERIC, "non-finite probe");
    mx = std::max(mx, h[i].x * h[i].x + h[i].y * h[i].y);
  }
  if (!(mx > 0.0)) return fail(MAGPIE_ERR_INVALID_ARG, "probe is identically zero");
  MG_HIP(hipMemcpyAsync(c->q64, h.data(), mm * sizeof(double2), hipMemcpyHostToDevice, c->stream));
  MG_HIP(hipStreamSynchronize(c->stream));
  c->u_given = false;
  rc = rebuild_levels(c);
  if (rc) return rc;
  c->has_probe = true;
  return MAGPIE_OK;
}

int magpie_set_regularization(magpie_ctx* c, double alpha, const double* u) {
  if (!c) return fail(MAGPIE_ERR_INVALID_ARG, "NULL context");
  if (!c->has_probe) return fail(MAGPIE_ERR_BAD_STATE, "set the probe first");
  int rc = set_dev(c);
  if (rc) return rc;
  if (u) {
    const size_t mm = (size_t)c->m * c->m;
    for (size_t i = 0; i < mm; ++i)
      if (!(u[i] >= 0.0) || !std::isfinite(u[i])) return fail(MAGPIE_ERR_INVALID_ARG, "u must be finite, >= 0");
    MG_HIP(hipMemcpyAsync(c->u0, u, mm * sizeof(double), hipMemcpyHostToDevice, c->stream));
    MG_HIP(hipStreamSynchronize(c->stream));
    c->u_given = true;
  } else {
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(MAGPIE_ERR_INVALID_ARG, "alpha must be finite, >= 0");
    c->alpha = alpha;
    c->u_given = false;
  }
  return rebuild_levels(c);
}

int magpie_set_positions(magpie_ctx* c, int n_pos, const int32_t* offsets) {
  if (!c || !offsets) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  if (n_pos < 1) return fail(MAGPIE_ERR_INVALID_ARG, "n_pos must be >= 1");
  for (int k = 0; k < n_pos; ++k) {
    const int r = offsets[2 * k], cc = offsets[2 * k + 1];
    if (r < 0 || r > c->nr - c->m || cc < 0 || cc > c->nc - c->m)
      return fail(MAGPIE_ERR_INVALID_ARG, "scan offset " + std::to_string(k) + " out of bounds");
  }
  int rc = set_dev(c);
  if (rc) return rc;
  MG_HIP(hipStreamSynchronize(c->stream));
  free_positions(c);
  const int m = c->m;
  rc = dev_alloc(&c->offs, n_pos);
  if (!rc) rc = dev_alloc(&c->sqrtd, (size_t)n_pos * m * m);
  if (!rc) rc = dev_alloc(&c->phi_step, n_pos);
  if (!rc) rc = dev_alloc(&c->phi_obj, n_pos);
  if (!rc) rc = dev_alloc(&c->gnorm, n_pos);
  if (!rc) rc = dev_alloc(&c->step_part, (size_t)n_pos * mg::MAX_WAVES);
  if (!rc) rc = dev_alloc(&c->obj_part, (size_t)n_pos * mg::MAX_WAVES);
  if (!rc) rc = dev_alloc(&c->gn_part, (size_t)n_pos * mg::MAX_WAVES);
  if (rc) {
    free_positions(c);
    return rc;
  }
  MG_HIP(hipMemcpyAsync(c->offs, offsets, (size_t)n_pos * sizeof(int2), hipMemcpyHostToDevice, c->stream));
  std::vector<double> nan((size_t)n_pos * mg::MAX_WAVES, std::nan(""));
  MG_HIP(hipMemcpyAsync(c->step_part, nan.data(), nan.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  MG_HIP(hipStreamSynchronize(c->stream));
  c->h_offs.assign(offsets, offsets + 2 * (size_t)n_pos);
  c->n_pos = n_pos;
  rc = build_tiles(c);
  if (rc) {
    free_positions(c);
    return rc;
  }
  c->has_pos = true;
  return reset_phases(c);
}

int magpie_load_intensities(magpie_ctx* c, const float* d, int is_sqrt, int on_device) {
  if (!c || !d) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  if (!c->has_pos) return fail(MAGPIE_ERR_BAD_STATE, "set positions first");
  int rc = set_dev(c);
  if (rc) return rc;
  const size_t cnt = (size_t)c->n_pos * c->m * c->m;
  const float* src = d;
  float* tmp = nullptr;
  if (!on_device) {
    rc = dev_alloc(&tmp, cnt);
    if (rc) return rc;
    hipError_t e = hipMemcpyAsync(tmp, d, cnt * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) {
      dev_free(tmp);
      return fail(MAGPIE_ERR_HIP, "intensity upload failed");
    }
    src = tmp;
  }
  MG_HIP(hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
  hipError_t e = mg::launch_permute_sqrt(c->m, c->rb, c->n_pos, src, is_sqrt ? 1 : 0, c->sqrtd, c->flag, c->stream);
  int bad = 0;
  rc = (e == hipSuccess) ? read_flag(c, &bad) : fail(MAGPIE_ERR_HIP, "permute kernel launch failed");
  dev_free(tmp);
  if (rc) return rc;
  if (bad) {
    c->has_data = false;
    return fail(MAGPIE_ERR_NUMERIC, "intensities contain negative or non-finite values");
  }
  c->has_data = true;
  return reset_phases(c);
}

int magpie_set_object(magpie_ctx* c, const void* z, int dtype, int on_device) {
  if (!c || !z) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  if (dtype != MAGPIE_C64 && dtype != MAGPIE_C128) return fail(MAGPIE_ERR_INVALID_ARG, "bad dtype");
  int rc = set_dev(c);
  if (rc) return rc;
  const size_t n = (size_t)c->nr * c->nc;
  if (on_device) {
    if (dtype == MAGPIE_C64) {
      MG_HIP(hipMemcpyAsync(c->z, z, n * sizeof(float2), hipMemcpyDeviceToDevice, c->stream));
    } else {
      MG_HIP(mg::launch_convert_c128_c64((const double2*)z, c->z, n, c->stream));
    }
  } else {
    if (dtype == MAGPIE_C64) {
      MG_HIP(hipMemcpyAsync(c->z, z, n * sizeof(float2), hipMemcpyHostToDevice, c->stream));
      MG_HIP(hipStreamSynchronize(c->stream));
    } else {
      std::vector<float2> t(n);
      const double2* p = (const double2*)z;
      for (size_t i = 0; i < n; ++i) t[i] = make_float2((float)p[i].x, (float)p[i].y);
      MG_HIP(hipMemcpyAsync(c->z, t.data(), n * sizeof(float2), hipMemcpyHostToDevice, c->stream));
      MG_HIP(hipStreamSynchronize(c->stream));
    }
  }
  MG_HIP(hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
  MG_HIP(mg::launch_check_finite_c64(c->z, n, c->flag, c->stream));
  int bad = 0;
  rc = read_flag(c, &bad);
  if (rc) return rc;
  if (bad) return fail(MAGPIE_ERR_NUMERIC, "object contains non-finite values");
  return MAGPIE_OK;
}

// Checks and device buffers for minibatches of B positions and the records of
// rec_epochs epochs (staging, probe-step partials with the flag, position records
// and inverse permutations), grown as needed.
static int ensure_epoch_buffers(magpie_ctx* c, int n_epochs, int batch, size_t rec_epochs) {
  if (!c) return fail(MAGPIE_ERR_INVALID_ARG, "NULL context");
  if (!c->has_probe || !c->has_pos || !c->has_data)
    return fail(MAGPIE_ERR_BAD_STATE, "set probe, positions and intensities first");
  if (n_epochs < 0 || batch < 1) return fail(MAGPIE_ERR_INVALID_ARG, "n_epochs >= 0 and batch >= 1 required");
  int rc = set_dev(c);
  if (rc) return rc;
  const int N = c->n_pos, m = c->m;
  const int B = std::min(batch, N);
  const size_t need_stage = (size_t)B * m * m;
  if (need_stage > c->stage_cap) {
    MG_HIP(hipStreamSynchronize(c->stream));
    drop_graph(c);   // a captured epoch holds the old buffers' addresses
    dev_free(c->stage);
    // the probe-step partials are sized with the staging: reallocated on next use
    dev_free(c->pnum);
    dev_free(c->pden);
    dev_free(c->pmax);
    dev_free(c->pacc);
    c->pcap = 0;
    rc = dev_alloc(&c->stage, need_stage);
    if (rc) {
      c->stage_cap = 0;
      return rc;
    }
    c->stage_cap = need_stage;
  }
  const bool probe_step = (c->flags & MAGPIE_UPDATE_PROBE) != 0;
  if (probe_step && need_stage > c->pcap) {
    MG_HIP(hipStreamSynchronize(c->stream));
    drop_graph(c);
    dev_free(c->pnum);
    dev_free(c->pden);
    dev_free(c->pmax);
    dev_free(c->pacc);
    rc = dev_alloc(&c->pnum, need_stage);
    if (!rc) rc = dev_alloc(&c->pden, need_stage);
    if (!rc) rc = dev_alloc(&c->pmax, (size_t)B * mg::MAX_WAVES);
    if (!rc) rc = dev_alloc(&c->pacc, mg::probe_scratch_doubles(m, B));
    if (rc) {
      c->pcap = 0;
      return rc;
    }
    c->pcap = need_stage;
  }
  const size_t nrec = rec_epochs * (size_t)N;
  if (nrec > c->perm_cap) {
    MG_HIP(hipStreamSynchronize(c->stream));
    drop_graph(c);
    dev_free(c->posrec);
    dev_free(c->posx);
    dev_free(c->inv);
    rc = dev_alloc(&c->inv, nrec);
    if (!rc) rc = dev_alloc(&c->posrec, nrec);
    if (!rc) rc = dev_alloc(&c->posx, nrec);
    if (rc) {
      dev_free(c->inv);
      dev_free(c->posrec);
      dev_free(c->posx);
      c->perm_cap = 0;
      return rc;
    }
    c->perm_cap = nrec;
  }
  return MAGPIE_OK;
}

// Pinned host area for the records of `epochs` epochs in each of the two slots
// (inverse permutation, then 4 ints per position record in processing order and 4
// in workgroup order), grown as needed once both slots' uploads are done.
static int ensure_pinned(magpie_ctx* c, size_t epochs) {
  const size_t need = 2 * epochs * (size_t)c->n_pos * 9;
  if (need <= c->h_pin_cap) return MAGPIE_OK;
  for (int s = 0; s < 2; ++s)
    if (c->pin_pending[s]) {
      MG_HIP(hipEventSynchronize(c->pin_done[s]));
      c->pin_pending[s] = false;
    }
  if (c->h_pin) hipHostFree(c->h_pin);
  c->h_pin = nullptr;
  c->h_pin_cap = 0;
  if (hipHostMalloc((void**)&c->h_pin, need * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
    c->h_pin = nullptr;
    return fail(MAGPIE_ERR_OOM, "pinned host allocation failed");
  }
  c->h_pin_cap = need;
  return MAGPIE_OK;
}

// An explicit order [n_epochs][N] must hold a permutation of 0..N-1 per row.
static int check_orders(magpie_ctx* c, int n_epochs, const int32_t* order) {
  const int N = c->n_pos;
  c->h_seen.assign((size_t)N, 0);
  for (int e = 0; e < n_epochs; ++e) {
    const int32_t* p = order + (size_t)e * N;
    for (int i = 0; i < N; ++i) {
      const int k = p[i];
      if (k < 0 || k >= N || c->h_seen[(size_t)k] == e + 1)
        return fail(MAGPIE_ERR_INVALID_ARG, "order row " + std::to_string(e) + " is not a permutation");
      c->h_seen[(size_t)k] = e + 1;
    }
  }
  return MAGPIE_OK;
}

// Workgroup order of one minibatch's records (bt records of 4 ints, processing
// order) into `out`: (k, row, col, slot).  A launch's consecutive workgroups go to
// the GPU's eight XCDs in turn, and each XCD has its own L2.  The windows are
// bucketed by the 16 x 16 cells (side 2^cs) of their corners, the buckets taken
// along a Morton curve (slot order within a bucket), and the result cut into eight
// contiguous runs, run x going to the workgroups x, x + 8, x + 16, ...: the windows
// one L2 serves are neighbours, so their patches overlap.  Every staged update and
// every sum stays at its slot, so the results do not change.
static void workgroup_order(const int32_t* rec, int bt, int cs, int32_t* out, std::vector<int>& cnt,
                            std::vector<int>& sorted) {
  auto key = [&](int i) {
    const uint32_t y = std::min(15u, (uint32_t)rec[4 * i + 1] >> cs);
    const uint32_t x = std::min(15u, (uint32_t)rec[4 * i + 2] >> cs);
    uint32_t k = 0;
    for (int b = 0; b < 4; ++b) k |= (((x >> b) & 1u) << (2 * b)) | (((y >> b) & 1u) << (2 * b + 1));
    return (int)k;
  };
  cnt.assign(257, 0);
  sorted.resize((size_t)bt);
  for (int i = 0; i < bt; ++i) ++cnt[(size_t)key(i) + 1];
  for (int k = 0; k < 256; ++k) cnt[(size_t)k + 1] += cnt[(size_t)k];
  for (int i = 0; i < bt; ++i) sorted[(size_t)cnt[(size_t)key(i)]++] = i;
  const int q = bt / 8, r = bt % 8;
  for (int w = 0; w < bt; ++w) {
    const int x = w % 8, j = x * q + std::min(x, r) + w / 8;
    const int sl = sorted[(size_t)j];
    out[4 * w] = rec[4 * sl];
    out[4 * w + 1] = rec[4 * sl + 1];
    out[4 * w + 2] = rec[4 * sl + 2];
    out[4 * w + 3] = sl;
  }
}

// Inverse permutations and position records (k, row, col) in processing order of
// epochs e0 .. e0+ne-1 (permutations from `order`, already checked, or the
// library's seeded ones for epoch counter c->epoch_index + e), built in pinned
// slot `slot` (slot_epochs epochs wide) and uploaded to the device records from
// epoch offset dev_epoch; the slot's event marks the end of its upload.  With
// batch > 0 the records of its minibatches in workgroup order go to c->posx too.
static int fill_records(magpie_ctx* c, int e0, int ne, uint64_t seed, const int32_t* order, int slot,
                        size_t slot_epochs, size_t dev_epoch, hipStream_t s, int batch = 0) {
  const int N = c->n_pos;
  // a slot's region moves with its width: then both slots' uploads must be done
  for (int s = 0; s < 2; ++s)
    if (c->pin_pending[s] && (s == slot || slot_epochs != c->pin_width)) {
      MG_HIP(hipEventSynchronize(c->pin_done[s]));
      c->pin_pending[s] = false;
    }
  c->pin_width = slot_epochs;
  int32_t* hi = c->h_pin + (size_t)slot * slot_epochs * N * 9;
  int32_t* hr = hi + slot_epochs * N;
  int32_t* hx = hr + slot_epochs * N * 4;
  int cs = 0;   // cell side 2^cs: corners fall in a 16 x 16 grid of cells
  while (((std::max(c->nr, c->nc) - 1) >> cs) >= 16) ++cs;
  c->h_perm.resize((size_t)N);
  for (int e = 0; e < ne; ++e) {
    const int32_t* p;
    if (order) {
      p = order + (size_t)(e0 + e) * N;
    } else {
      fisher_yates(seed, c->epoch_index + (uint64_t)(e0 + e), N, c->h_perm.data());
      p = c->h_perm.data();
    }
    int32_t* q = hi + (size_t)e * N;
    int32_t* r = hr + (size_t)e * N * 4;
    for (int i = 0; i < N; ++i) {
      const int k = p[i];
      q[k] = i;
      r[4 * i] = k;
      r[4 * i + 1] = c->h_offs[2 * (size_t)k];
      r[4 * i + 2] = c->h_offs[2 * (size_t)k + 1];
      r[4 * i + 3] = 0;
    }
    if (batch > 0)
      for (int t0 = 0; t0 < N; t0 += batch)
        workgroup_order(r + 4 * (size_t)t0, std::min(batch, N - t0), cs, hx + ((size_t)e * N + t0) * 4, c->h_cnt,
                        c->h_sorted);
  }
  const size_t n = (size_t)ne * N;
  MG_HIP(hipMemcpyAsync(c->inv + dev_epoch * N, hi, n * sizeof(int32_t), hipMemcpyHostToDevice, s));
  MG_HIP(hipMemcpyAsync(c->posrec + dev_epoch * N, hr, n * sizeof(int4), hipMemcpyHostToDevice, s));
  if (batch > 0) MG_HIP(hipMemcpyAsync(c->posx + dev_epoch * N, hx, n * sizeof(int4), hipMemcpyHostToDevice, s));
  MG_HIP(hipEventRecord(c->pin_done[slot], s));
  c->pin_pending[slot] = true;
  return MAGPIE_OK;
}

// Buffers, checks and the records of all n_epochs epochs at once (graph
// capture, multi-context rounds and single minibatches read them by epoch).
static int prepare_epochs(magpie_ctx* c, int n_epochs, int batch, uint64_t seed, const int32_t* order) {
  int rc = ensure_epoch_buffers(c, n_epochs, batch, (size_t)n_epochs);
  if (!rc && order) rc = check_orders(c, n_epochs, order);
  if (!rc) rc = ensure_pinned(c, (size_t)n_epochs);
  if (!rc) rc = fill_records(c, 0, n_epochs, seed, order, 0, (size_t)n_epochs, 0, c->stream);
  return rc;
}

}  // extern "C"

// Launches n_epochs prepared epochs of minibatch size B (the first
// batches_per_epoch minibatches of each; the rest are not run) on the buffers
// `buf` (the context's own, or the caller-free scratch of the no-allocation entry
// point, which passes allow_graph = false and has timing off).
int mgrt::launch_epochs(magpie_ctx* c, int n_epochs, int B, int batches_per_epoch, bool allow_graph,
                        const EpochBuffers& buf) {
  const int N = c->n_pos, m = c->m;
  const int nbatch = std::min((N + B - 1) / B, batches_per_epoch);
  const bool probe_step = (c->flags & MAGPIE_UPDATE_PROBE) != 0;

  mg::StepArgs sa{};
  sa.z = c->z;
  sa.n_rows = c->nr;
  sa.n_cols = c->nc;
  sa.q = c->qf;
  sa.qtab = c->qtab;
  sa.qspec = c->qspec;
  sa.sqrtd = c->sqrtd;
  sa.offs = c->offs;
  sa.stage = buf.stage;
  sa.u0f = c->u0f;
  sa.lvl = c->lvl;
  sa.levels = c->L;
  sa.lvl_a_off = c->lvl_a_off;
  sa.phi_part = c->step_part;
  sa.phase = (c->flags & MAGPIE_PHASE_RECYCLE) ? c->phase : nullptr;
  // a minibatch that fits in one workgroup per compute unit: stage with device
  // scope (see StepArgs::stage_wt)
  sa.stage_wt = (B <= c->n_cu) ? 1 : 0;
  if (probe_step) {
    sa.probe_num = c->pnum;
    sa.probe_den = c->pden;
    sa.probe_max = c->pmax;
  }
  // Alternating probe step: after the minibatch's object update a second pass of
  // the step kernel forms the probe partials at the new object (its staged
  // object update is not used, and it neither records Phi_k nor visits the
  // phase store).
  const bool alternate = probe_step && (c->flags & MAGPIE_PROBE_ALTERNATE);
  mg::StepArgs sp = sa;
  if (alternate) {
    sa.probe_num = nullptr;
    sa.probe_den = nullptr;
    sa.probe_max = nullptr;
    sp.phi_part = nullptr;
    sp.phase = nullptr;
  }
  auto probe_pass = [&]() -> hipError_t {
    sp.pos = sa.pos;
    sp.posx = sa.posx;
    sp.count = sa.count;
    sp.epoch = sa.epoch;
    sp.epoch_stride = sa.epoch_stride;
    return mg::launch_step(m, c->rb, mg::MODE_STEP, sp, c->stream);
  };
  const int nw = mg::step_waves(m, c->rb);
  // probe step after a minibatch's accumulation: apply, then rebuild the hierarchy
  auto probe_tail = [&](int count) -> hipError_t {
    hipError_t e =
        mg::launch_probe_apply(m, count, nw, c->pnum, c->pden, c->pmax, c->beta, c->q64, c->pacc, c->stream);
    if (e == hipSuccess)
      e = mg::launch_level_constants(c->m, c->L, c->alpha, c->u_given ? 1 : 0, c->q64, c->u0, c->w0, c->w0f,
                                     c->u0f, c->qf, c->lvl, c->lvl_a_off, c->scr_q, c->scr_u, c->rb, c->qtab,
                                     c->qspec, c->spec_tmp, c->stream);
    return e;
  };
  mg::AccumArgs aa{};
  aa.z = c->z;
  aa.n_rows = c->nr;
  aa.n_cols = c->nc;
  aa.m = m;
  aa.tiles_x = c->tiles_x;
  aa.box_x0 = c->box_x0;
  aa.box_y0 = c->box_y0;
  aa.box_nx = c->box_nx;
  aa.tile_ptr = c->tile_ptr;
  aa.tile_ent = c->tile_ent;
  aa.batch = B;
  aa.stage = buf.stage;
  aa.offs = c->offs;
  aa.w0f = c->w0f;
  const int n_tiles = c->box_nx * c->box_ny;
  aa.n_tiles = n_tiles;
  // small minibatches: each tile screens the minibatch's own records
  const bool scan = B <= mg::ACC_SCAN_MAX;
  const bool use_graph = allow_graph && !c->timing && (c->flags & MAGPIE_GRAPH);
  if (use_graph) {
    const void* key[4] = {buf.posrec, buf.inv, buf.stage, c->pnum};
    if (c->g_rb != c->rb || c->g_th != c->th) drop_graph(c);
    if (!c->gexec || c->g_batch != B || std::memcmp(key, c->g_key, sizeof(key)) != 0) {
      drop_graph(c);
      hipGraph_t graph = nullptr;
      MG_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
      hipError_t ce = hipSuccess;
      sa.epoch = c->epoch_ctr;
      sa.epoch_stride = N;
      aa.epoch = c->epoch_ctr;
      aa.epoch_stride = N;
      aa.inv = buf.inv;
      for (int t = 0; t < nbatch && ce == hipSuccess; ++t) {
        sa.pos = buf.posrec + (size_t)t * B;
        sa.count = std::min(B, N - t * B);
        ce = mg::launch_step(m, c->rb, mg::MODE_STEP, sa, c->stream);
        aa.batch_index = t;
        aa.pos = scan ? sa.pos : nullptr;
        aa.count = sa.count;
        if (ce == hipSuccess) ce = mg::launch_accumulate(aa, c->th, n_tiles, c->stream);
        if (ce == hipSuccess && alternate) ce = probe_pass();
        if (ce == hipSuccess && probe_step) ce = probe_tail(sa.count);
      }
      if (ce == hipSuccess) ce = mg::launch_advance_counter(c->epoch_ctr, c->stream);
      hipError_t ee = hipStreamEndCapture(c->stream, &graph);
      if (ce != hipSuccess || ee != hipSuccess) {
        if (graph) hipGraphDestroy(graph);
        return fail(MAGPIE_ERR_HIP, std::string("epoch graph capture failed: ") +
                                        hipGetErrorString(ce != hipSuccess ? ce : ee));
      }
      hipError_t ie = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
      hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        c->gexec = nullptr;
        return fail(MAGPIE_ERR_HIP, std::string("epoch graph instantiate failed: ") + hipGetErrorString(ie));
      }
      c->g_batch = B;
      c->g_rb = c->rb;
      c->g_th = c->th;
      std::memcpy(c->g_key, key, sizeof(key));
    }
    MG_HIP(mg::launch_set_counter(c->epoch_ctr, 0, c->stream));
    for (int e = 0; e < n_epochs; ++e) MG_HIP(hipGraphLaunch(c->gexec, c->stream));
    return MAGPIE_OK;
  }
  for (int e = 0; e < n_epochs; ++e) {
    for (int t = 0; t < nbatch; ++t) {
      sa.pos = buf.posrec + (size_t)e * N + (size_t)t * B;
      sa.posx = buf.posx ? buf.posx + (size_t)e * N + (size_t)t * B : nullptr;
      sa.count = std::min(B, N - t * B);
      int ti = timed_slot(c, 0, sa.count);
      MG_HIP(mg::launch_step(m, c->rb, mg::MODE_STEP, sa, c->stream, ti >= 0 ? c->timed[ti].a : nullptr,
                             ti >= 0 ? c->timed[ti].b : nullptr));
      aa.inv = buf.inv + (size_t)e * N;
      aa.batch_index = t;
      aa.pos = scan ? sa.pos : nullptr;
      aa.count = sa.count;
      ti = timed_slot(c, 1, 0);
      MG_HIP(mg::launch_accumulate(aa, c->th, n_tiles, c->stream, ti >= 0 ? c->timed[ti].a : nullptr,
                                   ti >= 0 ? c->timed[ti].b : nullptr));
      if (alternate) MG_HIP(probe_pass());
      if (probe_step) MG_HIP(probe_tail(sa.count));
    }
  }
  return MAGPIE_OK;
}

extern "C" {

int magpie_run_epochs(magpie_ctx* c, int n_epochs, int batch, uint64_t seed, const int32_t* order) {
  if (!c) return fail(MAGPIE_ERR_INVALID_ARG, "NULL context");
  if (c->flags & MAGPIE_PERSISTENT) {
    // the work-queue launch of the multi-context runs, with this context alone
    if (order) return fail(MAGPIE_ERR_UNSUPPORTED, "MAGPIE_PERSISTENT runs draw their own orders (seed)");
    if (batch < 1) return fail(MAGPIE_ERR_INVALID_ARG, "batch >= 1 required");
    return magpie_run_epochs_multi(&c, 1, n_epochs, &batch, seed);
  }
  if (n_epochs == 0 && batch >= 1) return MAGPIE_OK;
  const bool use_graph = !c->timing && (c->flags & MAGPIE_GRAPH);
  int rc;
  if (use_graph) {
    rc = prepare_epochs(c, n_epochs, batch, seed, order);
    if (rc) return rc;
    const int B = std::min(batch, c->n_pos);
    rc = launch_epochs(c, n_epochs, B, (c->n_pos + B - 1) / B, true,
                       EpochBuffers{c->stage, c->posrec, c->inv, nullptr});
    if (rc) return rc;
    c->epoch_index += (uint64_t)n_epochs;
    return MAGPIE_OK;
  }
  // Direct launches, with the host's part pipelined: the records of the next chunk
  // of epochs are drawn and uploaded (two pinned slots, two device halves) while
  // the GPU runs the current chunk.  The first chunk is one epoch, so the first
  // launch waits for one epoch's records only.
  // (buffers sized for a whole chunk from the first call on, so later calls with
  // more epochs reuse them)
  constexpr int CH = 8;
  const size_t ch = (size_t)CH;
  rc = ensure_epoch_buffers(c, n_epochs, batch, 2 * ch);
  if (!rc && order) rc = check_orders(c, n_epochs, order);
  if (!rc) rc = ensure_pinned(c, ch);
  if (rc) return rc;
  const int N = c->n_pos;
  const int B = std::min(batch, N);
  // workgroup order for the 128-point plans, whose gathers are bound by the patches'
  // L2 misses (measured no faster at m = 64)
  const bool xorder = c->m >= 128;
  int chunk = 0;
  for (int e0 = 0; e0 < n_epochs; ++chunk) {
    const int ne = chunk == 0 ? 1 : std::min(CH, n_epochs - e0);
    const int slot = chunk & 1;
    rc = fill_records(c, e0, ne, seed, order, slot, ch, (size_t)slot * ch, c->stream, xorder ? B : 0);
    if (rc) return rc;
    const size_t off = (size_t)slot * ch * N;
    rc = launch_epochs(c, ne, B, (N + B - 1) / B, false,
                       EpochBuffers{c->stage, c->posrec + off, c->inv + off, xorder ? c->posx + off : nullptr});
    if (rc) return rc;
    e0 += ne;
  }
  c->epoch_index += (uint64_t)n_epochs;
  return MAGPIE_OK;
}

int magpie_run_minibatch(magpie_ctx* c, int count, const int32_t* positions) {
  if (!c) return fail(MAGPIE_ERR_INVALID_ARG, "NULL context");
  if (!c->has_probe || !c->has_pos || !c->has_data)
    return fail(MAGPIE_ERR_BAD_STATE, "set probe, positions and intensities first");
  if (!positions || count < 1 || count > c->n_pos)
    return fail(MAGPIE_ERR_INVALID_ARG, "positions must list 1 .. n_pos distinct positions");
  // one epoch whose permutation starts with the given positions (the rest follow in
  // ascending order and are not run)
  std::vector<int32_t> order;
  order.reserve((size_t)c->n_pos);
  std::vector<char> seen((size_t)c->n_pos, 0);
  for (int i = 0; i < count; ++i) {
    const int k = positions[i];
    if (k < 0 || k >= c->n_pos || seen[(size_t)k])
      return fail(MAGPIE_ERR_INVALID_ARG, "positions must be distinct indices in [0, n_pos)");
    seen[(size_t)k] = 1;
    order.push_back(k);
  }
  for (int k = 0; k < c->n_pos; ++k)
    if (!seen[(size_t)k]) order.push_back(k);
  int rc = prepare_epochs(c, 1, count, 0, order.data());
  if (rc) return rc;
  return launch_epochs(c, 1, count, 1, false, EpochBuffers{c->stage, c->posrec, c->inv, nullptr});
}

int magpie_objective(magpie_ctx* c, double* phi, double* grad_stat) {
  if (!c || !phi) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  if (!c->has_probe || !c->has_pos || !c->has_data)
    return fail(MAGPIE_ERR_BAD_STATE, "set probe, positions and intensities first");
  int rc = set_dev(c);
  if (rc) return rc;
  mg::StepArgs sa{};
  sa.z = c->z;
  sa.n_rows = c->nr;
  sa.n_cols = c->nc;
  sa.q = c->qf;
  sa.qtab = c->qtab;
  sa.qspec = c->qspec;
  sa.sqrtd = c->sqrtd;
  sa.offs = c->offs;
  sa.perm = nullptr;
  sa.count = c->n_pos;
  sa.u0f = c->u0f;
  sa.lvl = c->lvl;
  sa.levels = c->L;
  sa.lvl_a_off = c->lvl_a_off;
  sa.phi_part = c->obj_part;
  sa.gn_part = c->gn_part;
  const int nw = mg::step_waves(c->m, c->rb);
  MG_HIP(mg::launch_step(c->m, c->rb, mg::MODE_OBJECTIVE, sa, c->stream));
  MG_HIP(mg::launch_reduce_parts(c->obj_part, c->n_pos, nw, 0, c->phi_obj, c->red, c->stream));
  MG_HIP(mg::launch_reduce_parts(c->gn_part, c->n_pos, nw, 1, c->gnorm, c->red + 1, c->stream));
  double h[2];
  MG_HIP(hipMemcpyAsync(h, c->red, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  MG_HIP(hipStreamSynchronize(c->stream));
  if (!std::isfinite(h[0]) || !std::isfinite(h[1])) return fail(MAGPIE_ERR_NUMERIC, "non-finite objective");
  *phi = h[0];
  if (grad_stat) *grad_stat = h[1] / ((double)c->n_pos * c->m);
  return MAGPIE_OK;
}

int magpie_get_step_phi(magpie_ctx* c, double* phi_k) {
  if (!c || !phi_k) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  if (!c->has_pos) return fail(MAGPIE_ERR_BAD_STATE, "no positions");
  int rc = set_dev(c);
  if (rc) return rc;
  MG_HIP(mg::launch_reduce_parts(c->step_part, c->n_pos, mg::step_waves(c->m, c->rb), 0, c->phi_step, nullptr, c->stream));
  MG_HIP(hipMemcpyAsync(phi_k, c->phi_step, (size_t)c->n_pos * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  MG_HIP(hipStreamSynchronize(c->stream));
  return MAGPIE_OK;
}

static int copy_out_c64(magpie_ctx* c, const float2* src, size_t n, void* out, int dtype, int on_device) {
  if (dtype != MAGPIE_C64 && dtype != MAGPIE_C128) return fail(MAGPIE_ERR_INVALID_ARG, "bad dtype");
  if (on_device) {
    if (dtype == MAGPIE_C64) {
      MG_HIP(hipMemcpyAsync(out, src, n * sizeof(float2), hipMemcpyDeviceToDevice, c->stream));
    } else {
      MG_HIP(mg::launch_convert_c64_c128(src, (double2*)out, n, c->stream));
    }
    return MAGPIE_OK;
  }
  if (dtype == MAGPIE_C64) {
    MG_HIP(hipMemcpyAsync(out, src, n * sizeof(float2), hipMemcpyDeviceToHost, c->stream));
    MG_HIP(hipStreamSynchronize(c->stream));
  } else {
    std::vector<float2> t(n);
    MG_HIP(hipMemcpyAsync(t.data(), src, n * sizeof(float2), hipMemcpyDeviceToHost, c->stream));
    MG_HIP(hipStreamSynchronize(c->stream));
    double2* o = (double2*)out;
    for (size_t i = 0; i < n; ++i) o[i] = make_double2(t[i].x, t[i].y);
  }
  return MAGPIE_OK;
}

int magpie_get_object(magpie_ctx* c, void* out, int dtype, int on_device) {
  if (!c || !out) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  int rc = set_dev(c);
  if (rc) return rc;
  return copy_out_c64(c, c->z, (size_t)c->nr * c->nc, out, dtype, on_device);
}

int magpie_get_probe(magpie_ctx* c, void* out, int dtype, int on_device) {
  if (!c || !out) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  if (!c->has_probe) return fail(MAGPIE_ERR_BAD_STATE, "no probe set");
  int rc = set_dev(c);
  if (rc) return rc;
  return copy_out_c64(c, c->qf, (size_t)c->m * c->m, out, dtype, on_device);
}

int magpie_sync(magpie_ctx* c) {
  if (!c) return fail(MAGPIE_ERR_INVALID_ARG, "NULL context");
  int rc = set_dev(c);
  if (rc) return rc;
  MG_HIP(hipStreamSynchronize(c->stream));
  return MAGPIE_OK;
}

int magpie_set_flags(magpie_ctx* c, uint32_t flags, double beta) {
  if (!c) return fail(MAGPIE_ERR_INVALID_ARG, "NULL context");
  if (flags & ~(MAGPIE_UPDATE_PROBE | MAGPIE_GRAPH | MAGPIE_PHASE_RECYCLE | MAGPIE_PROBE_ALTERNATE |
                MAGPIE_PERSISTENT))
    return fail(MAGPIE_ERR_INVALID_ARG, "unknown flag");
  if ((flags & MAGPIE_PROBE_ALTERNATE) && !(flags & MAGPIE_UPDATE_PROBE))
    return fail(MAGPIE_ERR_INVALID_ARG, "MAGPIE_PROBE_ALTERNATE needs MAGPIE_UPDATE_PROBE");
  if (!(beta >= 0.0) || !std::isfinite(beta)) return fail(MAGPIE_ERR_INVALID_ARG, "beta must be finite, >= 0");
  int rc = set_dev(c);
  if (rc) return rc;
  if (((c->flags ^ flags) & (MAGPIE_UPDATE_PROBE | MAGPIE_PHASE_RECYCLE | MAGPIE_PROBE_ALTERNATE)) ||
      beta != c->beta)
    drop_graph(c);
  const bool recycle_on = (flags & MAGPIE_PHASE_RECYCLE) && !(c->flags & MAGPIE_PHASE_RECYCLE);
  const bool recycle_off = !(flags & MAGPIE_PHASE_RECYCLE) && (c->flags & MAGPIE_PHASE_RECYCLE);
  c->flags = flags;
  c->beta = beta;
  if (recycle_on || recycle_off) return reset_phases(c);
  return MAGPIE_OK;
}

int magpie_forward_model(magpie_ctx* c, const void* z, int z_on_device, float* d_out, int out_on_device) {
  if (!c || !z || !d_out) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  if (!c->has_probe || !c->has_pos) return fail(MAGPIE_ERR_BAD_STATE, "set probe and positions first");
  int rc = set_dev(c);
  if (rc) return rc;
  const size_t nz = (size_t)c->nr * c->nc;
  const size_t nd = (size_t)c->n_pos * c->m * c->m;
  float2* zt = nullptr;
  float* dt = nullptr;
  const float2* zsrc = (const float2*)z;
  if (!z_on_device) {
    rc = dev_alloc(&zt, nz);
    if (rc) return rc;
    if (hipMemcpyAsync(zt, z, nz * sizeof(float2), hipMemcpyHostToDevice, c->stream) != hipSuccess) {
      dev_free(zt);
      return fail(MAGPIE_ERR_HIP, "object upload failed");
    }
    zsrc = zt;
  }
  float* dst = d_out;
  if (!out_on_device) {
    rc = dev_alloc(&dt, nd);
    if (rc) {
      dev_free(zt);
      return rc;
    }
    dst = dt;
  }
  mg::StepArgs sa{};
  sa.z = zsrc;
  sa.n_rows = c->nr;
  sa.n_cols = c->nc;
  sa.q = c->qf;
  sa.qtab = c->qtab;
  sa.qspec = c->qspec;
  sa.offs = c->offs;
  sa.perm = nullptr;
  sa.count = c->n_pos;
  sa.d_out = dst;
  hipError_t e = mg::launch_step(c->m, c->rb, mg::MODE_FORWARD, sa, c->stream);
  if (e == hipSuccess && !out_on_device)
    e = hipMemcpyAsync(d_out, dt, nd * sizeof(float), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_free(zt);
  dev_free(dt);
  if (e != hipSuccess) return fail(MAGPIE_ERR_HIP, std::string("forward model: ") + hipGetErrorString(e));
  return MAGPIE_OK;
}

// Returns the recorded launches' events to the pool and forgets the records.
static void recycle_timed(magpie_ctx* c) {
  for (auto& t : c->timed) {
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->timed.clear();
}

int magpie_set_timing(magpie_ctx* c, int enable) {
  if (!c) return fail(MAGPIE_ERR_INVALID_ARG, "NULL context");
  if (enable) {
    // records start anew; events still pending on the stream are waited for first
    int rc = set_dev(c);
    if (rc) return rc;
    MG_HIP(hipStreamSynchronize(c->stream));
    recycle_timed(c);
  }
  c->timing = enable != 0;
  return MAGPIE_OK;
}

int magpie_get_timing(magpie_ctx* c, double* step_ms, double* accum_ms, int64_t* step_launches,
                      int64_t* accum_launches, int64_t* positions) {
  if (!c || !step_ms || !accum_ms || !step_launches || !accum_launches || !positions)
    return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  int rc = set_dev(c);
  if (rc) return rc;
  MG_HIP(hipStreamSynchronize(c->stream));
  double ms[2] = {0.0, 0.0};
  int64_t nl[2] = {0, 0}, pos = 0;
  for (auto& t : c->timed) {
    float f = 0.0f;
    MG_HIP(hipEventElapsedTime(&f, t.a, t.b));   // on failure the records stay as they are
    ms[t.kind] += f;
    nl[t.kind] += 1;
    if (t.kind == 0) pos += t.count;
  }
  recycle_timed(c);
  *step_ms = ms[0];
  *accum_ms = ms[1];
  *step_launches = nl[0];
  *accum_launches = nl[1];
  *positions = pos;
  return MAGPIE_OK;
}

int magpie_get_launch_times(magpie_ctx* c, int kind, double* us, int32_t* positions, int cap) {
  if (!c || kind < 0 || kind > 1 || cap < 0 || (cap > 0 && (!us || !positions)))
    return fail(MAGPIE_ERR_INVALID_ARG, "bad argument");
  int rc = set_dev(c);
  if (rc) return rc;
  MG_HIP(hipStreamSynchronize(c->stream));
  int n = 0;
  for (auto& t : c->timed) {
    if (t.kind != kind) continue;
    if (n < cap) {
      float f = 0.0f;
      MG_HIP(hipEventElapsedTime(&f, t.a, t.b));
      us[n] = 1e3 * (double)f;
      positions[n] = t.count;
    }
    ++n;
  }
  return n;
}

int magpie_list_plans(int m, int32_t* threads_per_transform, int cap) {
  int tmp[8];
  const int n = mg::plans_for(m, tmp, 8);
  if (n == 0) return fail(MAGPIE_ERR_UNSUPPORTED, "no plan for this m");
  if (threads_per_transform)
    for (int i = 0; i < n && i < cap; ++i) threads_per_transform[i] = tmp[i];
  return n;
}

int magpie_get_tuning(magpie_ctx* c, int* threads_per_transform, int* tile_rows) {
  if (!c || !threads_per_transform || !tile_rows) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  *threads_per_transform = c->rb;
  *tile_rows = c->th;
  return MAGPIE_OK;
}

int magpie_set_tuning(magpie_ctx* c, int threads_per_transform, int tile_rows) {
  if (!c) return fail(MAGPIE_ERR_INVALID_ARG, "NULL context");
  const int rb = threads_per_transform ? threads_per_transform : c->rb;
  const int th = tile_rows ? tile_rows : c->th;
  if (!mg::plan_valid(c->m, rb)) return fail(MAGPIE_ERR_UNSUPPORTED, "no such FFT plan for this m");
  if (!mg::tile_valid(th)) return fail(MAGPIE_ERR_UNSUPPORTED, "tile rows must be 8, 16 or 32");
  int rc = set_dev(c);
  if (rc) return rc;
  if (rb != c->rb) {
    if (c->has_data) {
      // move sqrt(d) from the old plan's order to the new one through natural order
      const size_t cnt = (size_t)c->n_pos * c->m * c->m;
      float* nat = nullptr;
      rc = dev_alloc(&nat, cnt);
      if (rc) return rc;
      hipError_t e = mg::launch_unpermute_sqrt(c->m, c->rb, c->n_pos, c->sqrtd, nat, c->stream);
      if (e == hipSuccess) e = hipMemsetAsync(c->flag, 0, sizeof(int), c->stream);
      if (e == hipSuccess) e = mg::launch_permute_sqrt(c->m, rb, c->n_pos, nat, 1, c->sqrtd, c->flag, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      dev_free(nat);
      if (e != hipSuccess) return fail(MAGPIE_ERR_HIP, std::string("re-layout of sqrt(d): ") + hipGetErrorString(e));
    }
    c->rb = rb;
    if (c->has_probe) {
      rc = rebuild_levels(c);   // the probe table follows the plan's thread order
      if (rc) return rc;
    }
    if (c->has_pos) {
      std::vector<double> nan((size_t)c->n_pos * mg::MAX_WAVES, std::nan(""));
      MG_HIP(hipMemcpy(c->step_part, nan.data(), nan.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    drop_graph(c);
  }
  if (th != c->th) {
    c->th = th;
    if (c->has_pos) {
      rc = build_tiles(c);
      if (rc) return rc;
    }
    drop_graph(c);
  }
  return MAGPIE_OK;
}

int magpie_autotune(magpie_ctx* c, int batch, int trial_epochs, double* step_us, double* accum_us) {
  if (!c) return fail(MAGPIE_ERR_INVALID_ARG, "NULL context");
  if (!c->has_probe || !c->has_pos || !c->has_data)
    return fail(MAGPIE_ERR_BAD_STATE, "set probe, positions and intensities first");
  if (batch < 1 || trial_epochs < 1) return fail(MAGPIE_ERR_INVALID_ARG, "batch and trial_epochs must be >= 1");
  int rc = set_dev(c);
  if (rc) return rc;
  // the trials run real epochs: keep the object, epoch counter and flags, restore them after
  const size_t nz = (size_t)c->nr * c->nc;
  float2* zsave = nullptr;
  rc = dev_alloc(&zsave, nz);
  if (rc) return rc;
  MG_HIP(hipMemcpyAsync(zsave, c->z, nz * sizeof(float2), hipMemcpyDeviceToDevice, c->stream));
  const uint64_t ep = c->epoch_index;
  const uint32_t flags = c->flags;
  const bool timing = c->timing;
  // trials leave the probe and the phase store alone
  c->flags = flags & ~(MAGPIE_UPDATE_PROBE | MAGPIE_PHASE_RECYCLE | MAGPIE_PROBE_ALTERNATE);
  c->timing = true;
  double best_step = 1e300, best_acc = 1e300;
  int best_rb = c->rb, best_th = c->th;
  auto trial = [&](double* s_us, double* a_us) -> int {
    double s1, a1;
    int64_t sl, al, np;
    // one untimed epoch first: a kernel's first launch also loads its code
    c->timing = false;
    int r = magpie_run_epochs(c, 1, batch, 0x5eedull, nullptr);
    c->timing = true;
    if (!r) r = magpie_get_timing(c, &s1, &a1, &sl, &al, &np);   // reset
    if (!r) r = magpie_run_epochs(c, trial_epochs, batch, 0x5eedull, nullptr);
    if (!r) r = magpie_get_timing(c, &s1, &a1, &sl, &al, &np);
    if (!r) {
      *s_us = s1 * 1e3 / std::max<int64_t>(1, sl);
      *a_us = a1 * 1e3 / std::max<int64_t>(1, al);
    }
    return r;
  };
  int rbs[8];
  const int nplans = mg::plans_for(c->m, rbs, 8);
  for (int i = 0; i < nplans && !rc; ++i) {
    rc = magpie_set_tuning(c, rbs[i], 0);
    double su = 0, au = 0;
    if (!rc) rc = trial(&su, &au);
    if (!rc && su < best_step) {
      best_step = su;
      best_rb = rbs[i];
    }
  }
  const int ths[3] = {8, 16, 32};
  for (int i = 0; i < 3 && !rc; ++i) {
    rc = magpie_set_tuning(c, best_rb, ths[i]);
    double su = 0, au = 0;
    if (!rc) rc = trial(&su, &au);
    if (!rc && au < best_acc) {
      best_acc = au;
      best_th = ths[i];
    }
  }
  c->timing = timing;
  c->flags = flags;
  if (!rc) rc = magpie_set_tuning(c, best_rb, best_th);
  hipError_t e = hipMemcpyAsync(c->z, zsave, nz * sizeof(float2), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_free(zsave);
  c->epoch_index = ep;
  if (rc) return rc;
  if (e != hipSuccess) return fail(MAGPIE_ERR_HIP, "autotune restore failed");
  if (step_us) *step_us = best_step;
  if (accum_us) *accum_us = best_acc;
  return MAGPIE_OK;
}

int magpie_autotune_batch(magpie_ctx* c, const int32_t* candidates, int n_candidates, int trial_epochs,
                          int32_t* best_batch, double* rates) {
  if (!c) return fail(MAGPIE_ERR_INVALID_ARG, "NULL context");
  if (!candidates || n_candidates < 1 || !best_batch || trial_epochs < 1)
    return fail(MAGPIE_ERR_INVALID_ARG, "candidates, n_candidates >= 1, trial_epochs >= 1 and best_batch required");
  for (int i = 0; i < n_candidates; ++i)
    if (candidates[i] < 1) return fail(MAGPIE_ERR_INVALID_ARG, "minibatch candidates must be >= 1");
  if (!c->has_probe || !c->has_pos || !c->has_data)
    return fail(MAGPIE_ERR_BAD_STATE, "set probe, positions and intensities first");
  int rc = set_dev(c);
  if (rc) return rc;
  // buffers for the largest candidate first, so that no trial allocates inside its timing
  int bmax = 1;
  for (int i = 0; i < n_candidates; ++i) bmax = std::max(bmax, candidates[i]);
  rc = ensure_epoch_buffers(c, trial_epochs, bmax, 16);
  if (!rc) rc = ensure_pinned(c, 8);
  if (rc) return rc;
  const size_t nz = (size_t)c->nr * c->nc;
  float2* zsave = nullptr;
  rc = dev_alloc(&zsave, nz);
  if (rc) return rc;
  const uint64_t ep = c->epoch_index;
  const bool timing = c->timing;
  c->timing = false;
  hipError_t e = hipMemcpyAsync(zsave, c->z, nz * sizeof(float2), hipMemcpyDeviceToDevice, c->stream);
  double phi0 = 0.0;
  if (e != hipSuccess) rc = fail(MAGPIE_ERR_HIP, "autotune_batch save failed");
  if (!rc) rc = magpie_objective(c, &phi0, nullptr);
  double best_rate = -HUGE_VAL;
  int best = candidates[0];
  for (int i = 0; i < n_candidates && !rc; ++i) {
    e = hipMemcpyAsync(c->z, zsave, nz * sizeof(float2), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      rc = fail(MAGPIE_ERR_HIP, "autotune_batch restore failed");
      break;
    }
    c->epoch_index = ep;
    const auto t0 = std::chrono::steady_clock::now();
    rc = magpie_run_epochs(c, trial_epochs, candidates[i], 0x5eedull, nullptr);
    if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(MAGPIE_ERR_HIP, "autotune_batch run failed");
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    double phi1 = 0.0;
    if (!rc) rc = magpie_objective(c, &phi1, nullptr);
    if (rc) break;
    const double rate = (phi0 - phi1) / std::max(secs, 1e-9);
    if (rates) rates[i] = rate;
    if (rate > best_rate) {
      best_rate = rate;
      best = candidates[i];
    }
  }
  c->timing = timing;
  e = hipMemcpyAsync(c->z, zsave, nz * sizeof(float2), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_free(zsave);
  c->epoch_index = ep;
  if (rc) return rc;
  if (e != hipSuccess) return fail(MAGPIE_ERR_HIP, "autotune_batch restore failed");
  *best_batch = best;
  return MAGPIE_OK;
}

int magpie_run_epochs_multi(magpie_ctx* const* ctxs, int count, int n_epochs, const int* batch, uint64_t seed) {
  if (!ctxs || count < 1 || !batch) return fail(MAGPIE_ERR_INVALID_ARG, "contexts and batch sizes required");
  if (n_epochs < 0) return fail(MAGPIE_ERR_INVALID_ARG, "n_epochs >= 0 required");
  for (int i = 0; i < count; ++i) {
    if (!ctxs[i]) return fail(MAGPIE_ERR_INVALID_ARG, "NULL context in list");
    if (ctxs[i]->device != ctxs[0]->device) return fail(MAGPIE_ERR_INVALID_ARG, "contexts on different devices");
    if (ctxs[i]->flags & MAGPIE_UPDATE_PROBE)
      return fail(MAGPIE_ERR_UNSUPPORTED, "the probe step is not available in multi-context runs");
    if (ctxs[i]->flags & MAGPIE_PHASE_RECYCLE)
      return fail(MAGPIE_ERR_UNSUPPORTED, "phase recycling is not available in multi-context runs");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(MAGPIE_ERR_INVALID_ARG, "a context appears twice");
  }
  // MAGPIE_PERSISTENT: one work-queue launch per plan partition and chunk
  const bool queue = (ctxs[0]->flags & MAGPIE_PERSISTENT) != 0;
  for (int i = 1; i < count; ++i)
    if (((ctxs[i]->flags & MAGPIE_PERSISTENT) != 0) != queue)
      return fail(MAGPIE_ERR_INVALID_ARG, "MAGPIE_PERSISTENT must be set on every context of the run or on none");
  if (queue)
    for (int i = 0; i < count; ++i) {
      if (mg::qtile_rows(ctxs[i]->m, ctxs[i]->rb) == 0)
        return fail(MAGPIE_ERR_UNSUPPORTED, "the work-queue launch needs an FFT plan of at least 64 threads");
      if (std::min(batch[i], ctxs[i]->n_pos) > mg::ACC_SCAN_MAX)
        return fail(MAGPIE_ERR_UNSUPPORTED, "the work-queue launch takes minibatches of at most 256 positions");
    }
  if (n_epochs == 0) return MAGPIE_OK;
  magpie_ctx* c0 = ctxs[0];
  int rc = set_dev(c0);
  if (rc) return rc;
  hipStream_t st = c0->stream;
  // Epochs run in chunks of up to CH (the first chunk one epoch): the records and
  // round descriptors of a chunk are built on the host and uploaded (two pinned
  // and two device slots) while the GPU runs the previous chunk, and no buffer
  // grows with the number of epochs.
  constexpr int CH = 8;
  for (int i = 0; i < count; ++i) {
    rc = ensure_epoch_buffers(ctxs[i], n_epochs, batch[i], 2 * (size_t)CH);
    if (!rc) rc = ensure_pinned(ctxs[i], CH);
    if (rc) return rc;
  }
  std::vector<hipEvent_t> evs;
  auto join = [&](hipStream_t from, hipStream_t to) -> int {
    if (from == to) return MAGPIE_OK;
    hipEvent_t ev;
    MG_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    evs.push_back(ev);
    MG_HIP(hipEventRecord(ev, from));
    MG_HIP(hipStreamWaitEvent(to, ev, 0));
    return MAGPIE_OK;
  };
  auto cleanup = [&]() {
    for (auto ev : evs) hipEventDestroy(ev);
  };
  // every context's earlier work precedes this run
  for (int i = 1; i < count && !rc; ++i) rc = join(ctxs[i]->stream, st);
  if (rc) {
    cleanup();
    return rc;
  }
  // Partitions by FFT plan (m, rb).  Each runs its own rounds on a stream of its
  // own (the first on st, the others on the library's streams of this device, which
  // fork from st after each chunk's uploads and join it at the chunk's end), so the
  // partitions overlap and fill each other's launch tails.  Within a partition a
  // round pairs the t-th minibatches of its members: one step launch, then one
  // accumulation launch per tile height.
  struct Part {
    int m, rb;
    std::vector<int> members;
    std::vector<int> ths;                 // distinct tile heights of the members
    int R = 0;                            // rounds of the current chunk
    size_t desc0 = 0, pre0 = 0;           // offsets of its descriptors / running totals
    size_t pre_per_round = 0;
    size_t q0 = 0;                        // work queue: offset of its gpre / wait arrays (ints)
    hipStream_t stream = nullptr;
  };
  std::vector<Part> parts;
  for (int i = 0; i < count; ++i) {
    magpie_ctx* c = ctxs[i];
    Part* pp = nullptr;
    for (auto& p : parts)
      if (p.m == c->m && p.rb == c->rb) pp = &p;
    if (!pp) {
      parts.push_back(Part{c->m, c->rb, {}, {}});
      pp = &parts.back();
    }
    pp->members.push_back(i);
    if (std::find(pp->ths.begin(), pp->ths.end(), c->th) == pp->ths.end()) pp->ths.push_back(c->th);
  }
  // A plan of 1024-thread workgroups (one per CU) is split into two partitions of
  // about equal work (positions), so that one half's steps run while the other
  // half accumulates: 64-reconstruction workload 9.08 -> 9.58 M patterns/s, its 24
  // reconstructions with 128-point probes alone 4.84 -> 5.27 M.  (Splitting the
  // 512-thread plan's partition was slower: 19.9 -> 17.3 M on its 40 alone.)
  {
    std::vector<Part> split;
    for (auto& p : parts) {
      if (p.m * p.rb < 1024 || p.members.size() < 2) {
        split.push_back(p);
        continue;
      }
      std::vector<int> order(p.members);
      std::stable_sort(order.begin(), order.end(),
                       [&](int x, int y) { return ctxs[x]->n_pos > ctxs[y]->n_pos; });
      Part h[2] = {Part{p.m, p.rb, {}, {}}, Part{p.m, p.rb, {}, {}}};
      long long w[2] = {0, 0};
      for (int i : order) {
        const int k = w[1] < w[0] ? 1 : 0;
        h[k].members.push_back(i);
        w[k] += ctxs[i]->n_pos;
      }
      for (auto& q : h) {
        std::sort(q.members.begin(), q.members.end());
        for (int i : q.members)
          if (std::find(q.ths.begin(), q.ths.end(), ctxs[i]->th) == q.ths.end()) q.ths.push_back(ctxs[i]->th);
        split.push_back(q);
      }
    }
    parts.swap(split);
  }
  std::vector<int> B(count), nb(count);
  for (int i = 0; i < count; ++i) {
    B[i] = std::min(batch[i], ctxs[i]->n_pos);
    nb[i] = (ctxs[i]->n_pos + B[i] - 1) / B[i];
  }
  // work queue: every member's tiles at the plan's queue tile height; counters per
  // partition (done per member, then head), then the run's abort flag
  std::vector<size_t> qctr0(parts.size(), 0);
  long long wait_ticks = 0;
  size_t n_ctr = 0;
  if (queue) {
    for (size_t g = 0; g < parts.size(); ++g) {
      parts[g].ths.assign(1, mg::qtile_rows(parts[g].m, parts[g].rb));
      qctr0[g] = n_ctr;
      n_ctr += mg::queue_counter_ints((int)parts[g].members.size());
    }
    n_ctr += mg::QSLOT_STRIDE;   // the abort flag, on a line of its own
    if (c0->qctr_cap < n_ctr) {
      dev_free(c0->qctr);
      c0->qctr_cap = 0;
      rc = dev_alloc(&c0->qctr, n_ctr);
      if (rc) {
        cleanup();
        return rc;
      }
      c0->qctr_cap = n_ctr;
    }
    if (mg::clear_i32(c0->qctr, (int)n_ctr, st) != hipSuccess) {
      cleanup();
      return fail(MAGPIE_ERR_HIP, "work-queue counter clear failed");
    }
    // bound of one wait: 2 s of the GPU's constant wall clock (MAGPIE_QUEUE_WAIT_US overrides)
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c0->device) != hipSuccess || khz <= 0)
      khz = 100000;
    double us = 2e6;
    if (const char* env = std::getenv("MAGPIE_QUEUE_WAIT_US")) us = std::max(0.0, std::atof(env));
    wait_ticks = (long long)(us * 1e-3 * khz);
  }
  int* const q_abort = queue ? c0->qctr + (n_ctr - mg::QSLOT_STRIDE) : nullptr;
  std::vector<hipEvent_t> fork_ev(parts.size(), nullptr), join_ev(parts.size(), nullptr);
  for (size_t g = 0; g < parts.size() && !rc; ++g) {
    if (g == 0) {
      parts[g].stream = st;
      continue;
    }
    rc = side_stream(c0->device, (int)g - 1, &parts[g].stream);
    if (!rc && hipEventCreateWithFlags(&fork_ev[g], hipEventDisableTiming) != hipSuccess)
      rc = fail(MAGPIE_ERR_HIP, "hipEventCreate failed");
    if (fork_ev[g]) evs.push_back(fork_ev[g]);
    if (!rc && hipEventCreateWithFlags(&join_ev[g], hipEventDisableTiming) != hipSuccess)
      rc = fail(MAGPIE_ERR_HIP, "hipEventCreate failed");
    if (join_ev[g]) evs.push_back(join_ev[g]);
  }
  hipError_t e = hipSuccess;
  int chunk = 0;
  for (int e0 = 0; e0 < n_epochs && !rc && e == hipSuccess; ++chunk) {
    const int ne = chunk == 0 ? 1 : std::min(CH, n_epochs - e0);
    const int slot = chunk & 1;
    // records of every member for these epochs, uploaded on st into its device slot
    for (int i = 0; i < count && !rc; ++i)
      rc = fill_records(ctxs[i], e0, ne, seed, nullptr, slot, CH, (size_t)slot * CH, st);
    if (rc) break;
    // round descriptors of the chunk: per partition and round its members' step
    // descriptors, then their accumulation descriptors by tile height; running
    // totals: one block for the step launch, one per tile height (n_members + 1 ints)
    size_t n_desc = 0, n_pre = 0, n_q = 0;
    for (auto& p : parts) {
      p.R = 0;
      for (int i : p.members) p.R = std::max(p.R, ne * nb[i]);
      p.desc0 = n_desc;
      p.pre0 = n_pre;
      p.pre_per_round = (p.members.size() + 1) * (1 + p.ths.size());
      n_desc += (size_t)p.R * p.members.size();
      n_pre += (size_t)p.R * p.pre_per_round;
      p.q0 = n_q;
      if (queue) n_q += 2 * (2 * (size_t)p.R * p.members.size()) + 1;   // gpre (G + 1), wait (G)
    }
    const size_t off_a = (n_desc * sizeof(mg::StepArgs) + 255) & ~(size_t)255;
    const size_t off_p = (off_a + n_desc * sizeof(mg::AccumArgs) + 255) & ~(size_t)255;
    const size_t off_q = (off_p + n_pre * sizeof(int) + 255) & ~(size_t)255;
    const size_t bytes = off_q + n_q * sizeof(int);
    rc = multi_slot(c0, slot, bytes);
    if (rc) break;
    unsigned char* hbase = static_cast<unsigned char*>(c0->mdesc_host[slot]);
    unsigned char* dbase = c0->mdesc_dev[slot];
    mg::StepArgs* hs = reinterpret_cast<mg::StepArgs*>(hbase);
    mg::AccumArgs* ha = reinterpret_cast<mg::AccumArgs*>(hbase + off_a);
    int* hp = reinterpret_cast<int*>(hbase + off_p);
    std::fill(hp, hp + n_pre, 0);
    for (auto& p : parts) {
      const size_t nm = p.members.size();
      for (int r = 0; r < p.R; ++r) {
        mg::StepArgs* sd = hs + p.desc0 + (size_t)r * nm;
        mg::AccumArgs* ad = ha + p.desc0 + (size_t)r * nm;
        int* pre = hp + p.pre0 + (size_t)r * p.pre_per_round;
        for (size_t j = 0; j < nm; ++j) {
          const int i = p.members[j];
          magpie_ctx* c = ctxs[i];
          mg::StepArgs a{};
          a.z = c->z;
          a.n_rows = c->nr;
          a.n_cols = c->nc;
          a.q = c->qf;
          a.qtab = c->qtab;
          a.qspec = c->qspec;
          a.sqrtd = c->sqrtd;
          a.offs = c->offs;
          a.stage = c->stage;
          a.u0f = c->u0f;
          a.lvl = c->lvl;
          a.levels = c->L;
          a.lvl_a_off = c->lvl_a_off;
          a.phi_part = c->step_part;
          if (r < ne * nb[i]) {
            const int er = r / nb[i], t = r % nb[i];
            a.pos = c->posrec + ((size_t)slot * CH + er) * c->n_pos + (size_t)t * B[i];
            a.count = std::min(B[i], c->n_pos - t * B[i]);
          } else {
            a.count = 0;
          }
          pre[j + 1] = pre[j] + a.count;
          sd[j] = a;
        }
        size_t k = 0;
        for (size_t h = 0; h < p.ths.size(); ++h) {
          int* apre = pre + (nm + 1) * (1 + h);
          size_t jj = 0;
          for (size_t j = 0; j < nm; ++j) {
            const int i = p.members[j];
            magpie_ctx* c = ctxs[i];
            if (!queue && c->th != p.ths[h]) continue;
            mg::AccumArgs a{};
            a.z = c->z;
            a.n_rows = c->nr;
            a.n_cols = c->nc;
            a.m = c->m;
            a.tiles_x = c->tiles_x;
            a.box_x0 = c->box_x0;
            a.box_y0 = c->box_y0;
            a.box_nx = c->box_nx;
            a.tile_ptr = c->tile_ptr;
            a.tile_ent = c->tile_ent;
            a.stage = c->stage;
            a.offs = c->offs;
            a.w0f = c->w0f;
            a.batch = B[i];
            if (r < ne * nb[i]) {
              const int er = r / nb[i], t = r % nb[i];
              a.inv = c->inv + ((size_t)slot * CH + er) * c->n_pos;
              a.batch_index = t;
              a.n_tiles = c->box_nx * c->box_ny;
              if (queue) {   // the box at the queue's tile height (screened from the records)
                const int tq = p.ths[0];
                a.box_y0 = c->scan_r0 / tq;
                a.n_tiles = c->box_nx * (c->scan_r1 / tq - a.box_y0 + 1);
              }
              if (B[i] <= mg::ACC_SCAN_MAX) {
                a.pos = c->posrec + ((size_t)slot * CH + er) * c->n_pos + (size_t)t * B[i];
                a.count = std::min(B[i], c->n_pos - t * B[i]);
              }
            } else {
              a.inv = c->inv;
              a.n_tiles = 0;
            }
            apre[jj + 1] = apre[jj] + a.n_tiles;
            ad[k++] = a;
            ++jj;
          }
        }
      }
      if (queue) {
        // queue order: round r, steps of every member, then tiles of every member;
        // steps wait for the member's tiles of earlier rounds, tiles for its steps so far
        const size_t G = 2 * (size_t)p.R * nm;
        int* gpre = reinterpret_cast<int*>(hbase + off_q) + p.q0;
        int* wait = gpre + G + 1;
        std::vector<int> steps_so_far(nm, 0), tiles_before(nm, 0);
        gpre[0] = 0;
        for (int r = 0; r < p.R; ++r) {
          const mg::StepArgs* sd = hs + p.desc0 + (size_t)r * nm;
          const mg::AccumArgs* ad = ha + p.desc0 + (size_t)r * nm;
          for (size_t j = 0; j < nm; ++j) {
            const size_t g = (2 * (size_t)r) * nm + j;
            gpre[g + 1] = gpre[g] + sd[j].count;
            wait[g] = tiles_before[j];
            steps_so_far[j] += sd[j].count;
          }
          for (size_t j = 0; j < nm; ++j) {
            const size_t g = (2 * (size_t)r + 1) * nm + j;
            gpre[g + 1] = gpre[g] + ad[j].n_tiles;
            wait[g] = steps_so_far[j];
            tiles_before[j] += ad[j].n_tiles;
          }
        }
      }
    }
    e = hipMemcpyAsync(dbase, hbase, bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipEventRecord(c0->mdesc_done[slot], st);
    if (e != hipSuccess) break;
    c0->mdesc_pending[slot] = true;
    const mg::StepArgs* ds = reinterpret_cast<const mg::StepArgs*>(dbase);
    const mg::AccumArgs* da = reinterpret_cast<const mg::AccumArgs*>(dbase + off_a);
    const int* dp = reinterpret_cast<const int*>(dbase + off_p);
    // the other partitions start after the chunk's uploads
    for (size_t g = 1; g < parts.size() && e == hipSuccess; ++g) {
      e = hipEventRecord(fork_ev[g], st);
      if (e == hipSuccess) e = hipStreamWaitEvent(parts[g].stream, fork_ev[g], 0);
    }
    int R = 0;
    for (auto& p : parts) R = std::max(R, p.R);
    if (queue) R = 0;   // one work-queue launch per partition instead of the rounds below
    for (size_t g = 0; queue && g < parts.size() && e == hipSuccess; ++g) {
      const Part& p = parts[g];
      const size_t nm = p.members.size();
      const int* gpre = reinterpret_cast<const int*>(hbase + off_q) + p.q0;
      mg::QueueArgs q{};
      q.sdesc = ds + p.desc0;
      q.adesc = da + p.desc0;
      q.gpre = reinterpret_cast<const int*>(dbase + off_q) + p.q0;
      q.n_groups = (int)(2 * (size_t)p.R * nm);
      q.wait = q.gpre + q.n_groups + 1;
      q.n_members = (int)nm;
      q.total = gpre[q.n_groups];
      q.done = c0->qctr + qctr0[g];
      q.head = q.done + (size_t)2 * nm * mg::QSLOTS * mg::QSLOT_STRIDE;
      q.abort = q_abort;
      q.wait_ticks = wait_ticks;
      e = mg::clear_i32(q.done, (int)mg::queue_counter_ints((int)nm), p.stream);
      if (e == hipSuccess) e = mg::launch_queue(p.m, p.rb, q, c0->n_cu, p.stream);
    }
    for (int r = 0; r < R && e == hipSuccess; ++r) {
      for (size_t g = 0; g < parts.size() && e == hipSuccess; ++g) {
        const Part& p = parts[g];
        if (r >= p.R) continue;
        const size_t nm = p.members.size();
        const size_t dsc = p.desc0 + (size_t)r * nm;
        const size_t pre = p.pre0 + (size_t)r * p.pre_per_round;
        const int npat = hp[pre + nm];
        int ti = (npat > 0) ? timed_slot(c0, 0, npat) : -1;
        e = mg::launch_step_multi(p.m, p.rb, ds + dsc, dp + pre, (int)nm, npat, p.stream,
                                  ti >= 0 ? c0->timed[ti].a : nullptr, ti >= 0 ? c0->timed[ti].b : nullptr);
        size_t k = 0;
        for (size_t h = 0; h < p.ths.size() && e == hipSuccess; ++h) {
          size_t members_h = 0;
          for (int i : p.members) members_h += (ctxs[i]->th == p.ths[h]) ? 1 : 0;
          const size_t apre = pre + (nm + 1) * (1 + h);
          const int ntile = hp[apre + members_h];
          ti = (ntile > 0) ? timed_slot(c0, 1, 0) : -1;
          e = mg::launch_accumulate_multi(p.ths[h], da + dsc + k, dp + apre, (int)members_h, ntile, p.stream,
                                          ti >= 0 ? c0->timed[ti].a : nullptr, ti >= 0 ? c0->timed[ti].b : nullptr);
          k += members_h;
        }
      }
    }
    // the chunk ends on st (the chunk after next reuses this chunk's slots)
    for (size_t g = 1; g < parts.size() && e == hipSuccess; ++g) {
      e = hipEventRecord(join_ev[g], parts[g].stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, join_ev[g], 0);
    }
    e0 += ne;
  }
  if (!rc && e == hipSuccess) e = hipStreamSynchronize(st);
  if (!rc && e != hipSuccess) rc = fail(MAGPIE_ERR_HIP, std::string("multi-context run: ") + hipGetErrorString(e));
  if (!rc && queue) {
    int aborted = 0;
    e = hipMemcpy(&aborted, q_abort, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = fail(MAGPIE_ERR_HIP, std::string("multi-context run: ") + hipGetErrorString(e));
    else if (aborted)
      rc = fail(MAGPIE_ERR_HIP, "work-queue launch stopped (a wait for earlier items exceeded its bound); the "
                                "objects are left part-way through the run");
  }
  if (rc) {
    // a failed run returns only once nothing it queued still runs on the contexts' buffers
    for (auto& p : parts)
      if (p.stream) (void)hipStreamSynchronize(p.stream);
  }
  for (int i = 1; i < count && !rc; ++i) rc = join(st, ctxs[i]->stream);
  cleanup();
  if (rc) return rc;
  for (int i = 0; i < count; ++i) ctxs[i]->epoch_index += (uint64_t)n_epochs;
  return MAGPIE_OK;
}

int magpie_permutation(uint64_t seed, uint64_t epoch, int n, int32_t* out) {
  if (!out || n < 1) return fail(MAGPIE_ERR_INVALID_ARG, "n >= 1 and out required");
  fisher_yates(seed, epoch, n, out);
  return MAGPIE_OK;
}

int magpie_get_epoch_index(magpie_ctx* c, uint64_t* epoch_index) {
  if (!c || !epoch_index) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  *epoch_index = c->epoch_index;
  return MAGPIE_OK;
}

int magpie_set_epoch_index(magpie_ctx* c, uint64_t epoch_index) {
  if (!c) return fail(MAGPIE_ERR_INVALID_ARG, "NULL context");
  c->epoch_index = epoch_index;
  return MAGPIE_OK;
}

}  // extern "C"
