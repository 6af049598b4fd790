// Host runtime of the learned-start C ABI (include/magpie_learned.h): the
// coarse-object network (buffers, forward, loss, backward, Adam), the input
// map and object pyramid on a reconstruction context, and the learned start
// with its flat-start fallback.
#include "../../include/magpie_learned.h"

#include "cnn.h"
#include "context.h"

using namespace mgrt;

namespace {

constexpr int N_LAYERS = 5;
constexpr int WIDTH = 32;

template <typename T>
int grow(T** p, size_t* cap, size_t count) {
  if (*cap >= count && *p) return MAGPIE_OK;
  dev_free(*p);
  *cap = 0;
  int rc = dev_alloc(p, count);
  if (!rc) *cap = count;
  return rc;
}

}  // namespace

struct magpie_cnn {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int cin = 3, side = 0, max_batch = 0;
  bool bf16 = false;
  int64_t n = 0;
  int co[N_LAYERS], ci[N_LAYERS];
  int64_t off_w[N_LAYERS], off_b[N_LAYERS];
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  int64_t t = 0;
  void* wf[N_LAYERS] = {};
  void* wt[N_LAYERS] = {};
  float *x = nullptr, *a1 = nullptr, *a2 = nullptr, *a3 = nullptr, *a4 = nullptr, *y = nullptr, *dy = nullptr;
  float *f0 = nullptr, *f1 = nullptr, *l0 = nullptr, *l1 = nullptr;
  float* part = nullptr;
  double* lpart = nullptr;
  double* lsum = nullptr;
  float2* tgt = nullptr;
  float* mask = nullptr;
  float2* rot = nullptr;
  double2* ip_part = nullptr;
  int last_batch = 0;
  bool have_dy = false;
};

namespace {

int cnn_dev(magpie_cnn* net) {
  MG_HIP(hipSetDevice(net->device));
  return MAGPIE_OK;
}

int prep_weights(magpie_cnn* net) {
  for (int l = 0; l < N_LAYERS; ++l)
    MG_HIP(cnn::launch_prep_weights(net->p + net->off_w[l], net->wf[l], net->wt[l], net->co[l], net->ci[l], net->bf16,
                                    net->stream));
  return MAGPIE_OK;
}

int copy_in(void* dst, const void* src, size_t bytes, int on_device, hipStream_t s) {
  MG_HIP(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  if (!on_device) MG_HIP(hipStreamSynchronize(s));
  return MAGPIE_OK;
}

int copy_out(void* dst, const void* src, size_t bytes, int on_device, hipStream_t s) {
  MG_HIP(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  if (!on_device) MG_HIP(hipStreamSynchronize(s));
  return MAGPIE_OK;
}

// layer l: grad rows of the weight-gradient kernel summed into g
int layer_wgrad(magpie_cnn* net, int l, bool up, const float* in, const float* dout, int nb, int H, int W) {
  const int nwg = cnn::wgrad_workgroups(nb, H, W);
  if (nwg > cnn::WGRAD_MAX_WORKGROUPS) return fail(MAGPIE_ERR_HIP, "weight-gradient partials exceed their buffer");
  const int row = net->co[l] * net->ci[l] * 9 + net->co[l];
  MG_HIP(cnn::launch_wgrad(up, in, dout, net->part, nb, net->ci[l], net->co[l], H, W, net->stream));
  MG_HIP(cnn::launch_rows_sum(net->part, nwg, row, net->g + net->off_w[l], net->stream));
  return MAGPIE_OK;
}

bool pow2(int f) { return f >= 1 && (f & (f - 1)) == 0; }

int need_ctx_data(magpie_ctx* c) {
  if (!c->has_probe || !c->has_pos || !c->has_data)
    return fail(MAGPIE_ERR_BAD_STATE, "set probe, positions and intensities first");
  return MAGPIE_OK;
}

// input map into c->lrn_map (device), stream-ordered on the context's stream
int input_map_dev(magpie_ctx* c, int side) {
  int rc = need_ctx_data(c);
  if (rc) return rc;
  if (side < 1 || c->nr % side || c->nc % side)
    return fail(MAGPIE_ERR_INVALID_ARG, "side must divide the object's rows and columns");
  if (side > cnn::PHASE_MAX_SIDE) return fail(MAGPIE_ERR_UNSUPPORTED, "side must be at most 64");
  const size_t mm = (size_t)c->m * c->m;
  rc = grow(&c->lrn_sd, &c->lrn_sd_cap, (size_t)c->n_pos * mm);
  if (!rc) rc = grow(&c->lrn_stats, &c->lrn_stats_cap, (size_t)c->n_pos);
  if (!rc) rc = grow(&c->lrn_fine, &c->lrn_fine_cap, 3 * (size_t)c->nr * c->nc);
  if (!rc) rc = grow(&c->lrn_map, &c->lrn_map_cap, 4 * (size_t)side * side);
  if (!rc && !c->lrn_q) rc = dev_alloc(&c->lrn_q, 1);
  if (rc) return rc;
  MG_HIP(mg::launch_unpermute_sqrt(c->m, c->rb, c->n_pos, c->sqrtd, c->lrn_sd, c->stream));
  MG_HIP(cnn::launch_probe_norm(c->q64, c->m, c->lrn_q, c->stream));
  MG_HIP(cnn::launch_position_stats(c->lrn_sd, c->n_pos, c->m, c->lrn_q, c->lrn_stats, c->stream));
  MG_HIP(cnn::launch_map_fine(c->lrn_stats, c->q64, c->m, c->tile_ptr, c->tile_ent, c->tiles_x, mg::ACC_TILE_W, c->th,
                              c->nr, c->nc, c->lrn_fine, c->stream));
  MG_HIP(cnn::launch_pool(c->lrn_fine, c->nr, c->nc, c->nr / side, c->nc / side, c->lrn_map, c->stream));
  // channel 3: the phase the centre-of-mass channels (slopes of 2 pi f / m per
  // object pixel, f in DFT bins) integrate to, per map cell
  const size_t ss = (size_t)side * side;
  const double two_pi = 6.283185307179586;
  MG_HIP(cnn::launch_integrate_phase(c->lrn_map + ss, c->lrn_map + 2 * ss, side, two_pi * (c->nr / side) / c->m,
                                     two_pi * (c->nc / side) / c->m, c->lrn_map + 3 * ss, c->stream));
  return MAGPIE_OK;
}

int prolong_into_object(magpie_ctx* c, const void* coarse_dev, int side, int format) {
  const int f = c->nr / side;
  MG_HIP(cnn::launch_prolong_object(coarse_dev, format, side, side, f, c->z, c->nr, c->nc, c->stream));
  return MAGPIE_OK;
}

int check_object_finite(magpie_ctx* c) {
  MG_HIP(hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
  MG_HIP(mg::launch_check_finite_c64(c->z, (size_t)c->nr * c->nc, c->flag, c->stream));
  int bad = 0;
  int rc = read_flag(c, &bad);
  if (rc) return rc;
  return bad ? fail(MAGPIE_ERR_NUMERIC, "object contains non-finite values") : MAGPIE_OK;
}

}  // namespace

extern "C" {

int magpie_cnn_create(magpie_cnn** out, int in_ch, int width, int side, int max_batch, int weight_dtype, int device,
                      void* stream) {
  if (!out) return fail(MAGPIE_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (in_ch != 1 && in_ch != 3 && in_ch != 4) return fail(MAGPIE_ERR_UNSUPPORTED, "in_ch must be 1, 3 or 4");
  if (width != WIDTH) return fail(MAGPIE_ERR_UNSUPPORTED, "width must be 32");
  if (side < 2 || (side & 1)) return fail(MAGPIE_ERR_INVALID_ARG, "side must be even and >= 2");
  if (max_batch < 1) return fail(MAGPIE_ERR_INVALID_ARG, "max_batch >= 1 required");
  if (weight_dtype != MAGPIE_W_F32 && weight_dtype != MAGPIE_W_BF16)
    return fail(MAGPIE_ERR_INVALID_ARG, "weight_dtype must be MAGPIE_W_F32 or MAGPIE_W_BF16");
  int ndev = 0;
  MG_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(MAGPIE_ERR_INVALID_ARG, "no such device");
  magpie_cnn* net = new magpie_cnn();
  net->device = device;
  net->cin = in_ch;
  net->side = side;
  net->max_batch = max_batch;
  net->bf16 = weight_dtype == MAGPIE_W_BF16;
  const int cos[N_LAYERS] = {WIDTH, WIDTH, WIDTH, WIDTH, 2};
  const int cis[N_LAYERS] = {in_ch, WIDTH, WIDTH, WIDTH, WIDTH};
  int64_t off = 0;
  for (int l = 0; l < N_LAYERS; ++l) {
    net->co[l] = cos[l];
    net->ci[l] = cis[l];
    net->off_w[l] = off;
    off += (int64_t)cos[l] * cis[l] * 9;
    net->off_b[l] = off;
    off += cos[l];
  }
  net->n = off;
  int rc = cnn_dev(net);
  if (rc) {
    delete net;
    return rc;
  }
  if (stream) {
    net->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&net->stream, hipStreamNonBlocking) != hipSuccess) {
      delete net;
      return fail(MAGPIE_ERR_HIP, "hipStreamCreate failed");
    }
    net->own_stream = true;
  }
  const size_t B = (size_t)max_batch, S = side, S2 = 2 * (size_t)side;
  const size_t lo = B * WIDTH * S * S, hi = B * WIDTH * S2 * S2;
  const size_t wsz = net->bf16 ? sizeof(uint16_t) : sizeof(float);
  rc = dev_alloc(&net->p, (size_t)net->n);
  if (!rc) rc = dev_alloc(&net->g, (size_t)net->n);
  if (!rc) rc = dev_alloc(&net->m, (size_t)net->n);
  if (!rc) rc = dev_alloc(&net->v, (size_t)net->n);
  for (int l = 0; l < N_LAYERS && !rc; ++l) {
    const size_t cnt = (size_t)net->co[l] * net->ci[l] * 9 * wsz;
    rc = dev_alloc((char**)&net->wf[l], cnt);
    if (!rc) rc = dev_alloc((char**)&net->wt[l], cnt);
  }
  if (!rc) rc = dev_alloc(&net->x, B * in_ch * S * S);
  if (!rc) rc = dev_alloc(&net->a1, lo);
  if (!rc) rc = dev_alloc(&net->a2, lo);
  if (!rc) rc = dev_alloc(&net->l0, lo);
  if (!rc) rc = dev_alloc(&net->l1, lo);
  if (!rc) rc = dev_alloc(&net->a3, hi);
  if (!rc) rc = dev_alloc(&net->a4, hi);
  if (!rc) rc = dev_alloc(&net->f0, hi);
  if (!rc) rc = dev_alloc(&net->f1, hi);
  if (!rc) rc = dev_alloc(&net->y, B * 2 * S2 * S2);
  if (!rc) rc = dev_alloc(&net->dy, B * 2 * S2 * S2);
  if (!rc) rc = dev_alloc(&net->part, (size_t)cnn::WGRAD_MAX_WORKGROUPS * (WIDTH * WIDTH * 9 + WIDTH));
  if (!rc) rc = dev_alloc(&net->lpart, (size_t)cnn::cmse_blocks(max_batch, (int)(S2 * S2)));
  if (!rc) rc = dev_alloc(&net->lsum, 1);
  if (!rc) rc = dev_alloc(&net->tgt, B * S2 * S2);
  if (!rc) rc = dev_alloc(&net->mask, S2 * S2);
  if (!rc) rc = dev_alloc(&net->rot, B);
  if (!rc) rc = dev_alloc(&net->ip_part, B * (size_t)cnn::cmse_ip_blocks((int)(S2 * S2)));
  if (rc) {
    magpie_cnn_destroy(net);
    return rc;
  }
  if (hipMemsetAsync(net->p, 0, net->n * sizeof(float), net->stream) != hipSuccess ||
      hipMemsetAsync(net->m, 0, net->n * sizeof(float), net->stream) != hipSuccess ||
      hipMemsetAsync(net->v, 0, net->n * sizeof(float), net->stream) != hipSuccess ||
      hipMemsetAsync(net->g, 0, net->n * sizeof(float), net->stream) != hipSuccess) {
    magpie_cnn_destroy(net);
    return fail(MAGPIE_ERR_HIP, "parameter init failed");
  }
  rc = prep_weights(net);
  if (!rc && hipStreamSynchronize(net->stream) != hipSuccess) rc = fail(MAGPIE_ERR_HIP, "init sync failed");
  if (rc) {
    magpie_cnn_destroy(net);
    return rc;
  }
  *out = net;
  return MAGPIE_OK;
}

int magpie_cnn_destroy(magpie_cnn* net) {
  if (!net) return MAGPIE_OK;
  hipSetDevice(net->device);
  if (net->stream) hipStreamSynchronize(net->stream);
  dev_free(net->p);
  dev_free(net->g);
  dev_free(net->m);
  dev_free(net->v);
  for (int l = 0; l < N_LAYERS; ++l) {
    dev_free(net->wf[l]);
    dev_free(net->wt[l]);
  }
  dev_free(net->x);
  dev_free(net->a1);
  dev_free(net->a2);
  dev_free(net->a3);
  dev_free(net->a4);
  dev_free(net->y);
  dev_free(net->dy);
  dev_free(net->f0);
  dev_free(net->f1);
  dev_free(net->l0);
  dev_free(net->l1);
  dev_free(net->part);
  dev_free(net->lpart);
  dev_free(net->lsum);
  dev_free(net->tgt);
  dev_free(net->mask);
  dev_free(net->rot);
  dev_free(net->ip_part);
  if (net->own_stream && net->stream) hipStreamDestroy(net->stream);
  delete net;
  return MAGPIE_OK;
}

int magpie_cnn_num_params(const magpie_cnn* net, int64_t* n) {
  if (!net || !n) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  *n = net->n;
  return MAGPIE_OK;
}

int magpie_cnn_set_params(magpie_cnn* net, const float* params, int on_device) {
  if (!net || !params) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  int rc = cnn_dev(net);
  if (rc) return rc;
  if (!on_device) {
    for (int64_t i = 0; i < net->n; ++i)
      if (!std::isfinite(params[i])) return fail(MAGPIE_ERR_NUMERIC, "non-finite parameter");
  }
  rc = copy_in(net->p, params, net->n * sizeof(float), on_device, net->stream);
  if (rc) return rc;
  MG_HIP(hipMemsetAsync(net->m, 0, net->n * sizeof(float), net->stream));
  MG_HIP(hipMemsetAsync(net->v, 0, net->n * sizeof(float), net->stream));
  net->t = 0;
  return prep_weights(net);
}

int magpie_cnn_get_params(magpie_cnn* net, float* params, int on_device) {
  if (!net || !params) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  int rc = cnn_dev(net);
  if (rc) return rc;
  return copy_out(params, net->p, net->n * sizeof(float), on_device, net->stream);
}

int magpie_cnn_get_grads(magpie_cnn* net, float* grads, int on_device) {
  if (!net || !grads) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  int rc = cnn_dev(net);
  if (rc) return rc;
  return copy_out(grads, net->g, net->n * sizeof(float), on_device, net->stream);
}

int magpie_cnn_forward(magpie_cnn* net, const float* x, float* y, int nbatch, int on_device) {
  if (!net || !x) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  if (nbatch < 1 || nbatch > net->max_batch) return fail(MAGPIE_ERR_INVALID_ARG, "nbatch must be in [1, max_batch]");
  int rc = cnn_dev(net);
  if (rc) return rc;
  const int S = net->side, S2 = 2 * S;
  hipStream_t s = net->stream;
  rc = copy_in(net->x, x, (size_t)nbatch * net->cin * S * S * sizeof(float), on_device, s);
  if (rc) return rc;
  const bool bf = net->bf16;
  MG_HIP(cnn::launch_conv(WIDTH, false, 0, bf, net->x, net->wf[0], net->p + net->off_b[0], net->a1, nullptr, nbatch,
                          net->cin, S, S, s));
  MG_HIP(cnn::launch_conv(WIDTH, false, 0, bf, net->a1, net->wf[1], net->p + net->off_b[1], net->a2, nullptr, nbatch,
                          WIDTH, S, S, s));
  MG_HIP(cnn::launch_conv(WIDTH, true, 0, bf, net->a2, net->wf[2], net->p + net->off_b[2], net->a3, nullptr, nbatch,
                          WIDTH, S2, S2, s));
  MG_HIP(cnn::launch_conv(WIDTH, false, 0, bf, net->a3, net->wf[3], net->p + net->off_b[3], net->a4, nullptr, nbatch,
                          WIDTH, S2, S2, s));
  MG_HIP(cnn::launch_conv(2, false, 1, bf, net->a4, net->wf[4], net->p + net->off_b[4], net->y, nullptr, nbatch,
                          WIDTH, S2, S2, s));
  net->last_batch = nbatch;
  net->have_dy = false;
  if (y) return copy_out(y, net->y, (size_t)nbatch * 2 * S2 * S2 * sizeof(float), on_device, s);
  return MAGPIE_OK;
}

int magpie_cnn_loss(magpie_cnn* net, const void* target, const float* mask, int nbatch, int align_phase,
                    int on_device, double* loss) {
  if (!net || !target || !mask || !loss) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  if (nbatch != net->last_batch || nbatch < 1) return fail(MAGPIE_ERR_BAD_STATE, "run forward with this nbatch first");
  int rc = cnn_dev(net);
  if (rc) return rc;
  const int S2 = 2 * net->side, hw = S2 * S2;
  hipStream_t s = net->stream;
  rc = copy_in(net->tgt, target, (size_t)nbatch * hw * sizeof(float2), on_device, s);
  if (!rc) rc = copy_in(net->mask, mask, (size_t)hw * sizeof(float), on_device, s);
  if (rc) return rc;
  std::vector<float> hm(hw);
  MG_HIP(hipMemcpyAsync(hm.data(), net->mask, hw * sizeof(float), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  double msum = 0.0;
  for (float v : hm) {
    if (!(v >= 0.0f) || !std::isfinite(v)) return fail(MAGPIE_ERR_INVALID_ARG, "mask must be finite and >= 0");
    msum += v;
  }
  if (!(msum > 0.0)) return fail(MAGPIE_ERR_INVALID_ARG, "mask is all zero");
  const double inv = 1.0 / ((double)nbatch * msum);
  MG_HIP(cnn::launch_cmse(net->y, net->tgt, net->mask, align_phase ? net->rot : nullptr, net->ip_part, net->dy,
                          net->lpart, nbatch, hw, (float)inv, s));
  MG_HIP(cnn::launch_sum_f64(net->lpart, cnn::cmse_blocks(nbatch, hw), net->lsum, s));
  double h = 0.0;
  MG_HIP(hipMemcpyAsync(&h, net->lsum, sizeof(double), hipMemcpyDeviceToHost, s));
  MG_HIP(hipStreamSynchronize(s));
  *loss = h * inv;
  net->have_dy = true;
  return std::isfinite(*loss) ? MAGPIE_OK : fail(MAGPIE_ERR_NUMERIC, "non-finite loss");
}

int magpie_cnn_backward(magpie_cnn* net, const float* dy, int nbatch, int on_device) {
  if (!net) return fail(MAGPIE_ERR_INVALID_ARG, "NULL network");
  if (nbatch != net->last_batch || nbatch < 1) return fail(MAGPIE_ERR_BAD_STATE, "run forward with this nbatch first");
  if (!dy && !net->have_dy) return fail(MAGPIE_ERR_BAD_STATE, "no stored output gradient: pass dy or call loss");
  int rc = cnn_dev(net);
  if (rc) return rc;
  const int S = net->side, S2 = 2 * S, nb = nbatch;
  hipStream_t s = net->stream;
  if (dy) {
    rc = copy_in(net->dy, dy, (size_t)nb * 2 * S2 * S2 * sizeof(float), on_device, s);
    if (rc) return rc;
  }
  const bool bf = net->bf16;
  // layer 5: dy -> dW5, dp4 = (W5^T * dy) on a4 > 0
  rc = layer_wgrad(net, 4, false, net->a4, net->dy, nb, S2, S2);
  if (rc) return rc;
  MG_HIP(cnn::launch_conv(WIDTH, false, 2, bf, net->dy, net->wt[4], nullptr, net->f0, net->a4, nb, 2, S2, S2, s));
  // layer 4
  rc = layer_wgrad(net, 3, false, net->a3, net->f0, nb, S2, S2);
  if (rc) return rc;
  MG_HIP(cnn::launch_conv(WIDTH, false, 2, bf, net->f0, net->wt[3], nullptr, net->f1, net->a3, nb, WIDTH, S2, S2, s));
  // layer 3 (input read through the upsampling)
  rc = layer_wgrad(net, 2, true, net->a2, net->f1, nb, S2, S2);
  if (rc) return rc;
  MG_HIP(cnn::launch_conv(WIDTH, false, 3, bf, net->f1, net->wt[2], nullptr, net->f0, nullptr, nb, WIDTH, S2, S2, s));
  MG_HIP(cnn::launch_up_backward_mask(net->f0, net->a2, net->l0, nb, WIDTH, S, S, s));
  // layer 2
  rc = layer_wgrad(net, 1, false, net->a1, net->l0, nb, S, S);
  if (rc) return rc;
  MG_HIP(cnn::launch_conv(WIDTH, false, 2, bf, net->l0, net->wt[1], nullptr, net->l1, net->a1, nb, WIDTH, S, S, s));
  // layer 1
  return layer_wgrad(net, 0, false, net->x, net->l1, nb, S, S);
}

int magpie_cnn_adam_step(magpie_cnn* net, float lr, float beta1, float beta2, float eps) {
  if (!net) return fail(MAGPIE_ERR_INVALID_ARG, "NULL network");
  if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return fail(MAGPIE_ERR_INVALID_ARG, "need lr > 0, 0 <= beta < 1, eps > 0");
  int rc = cnn_dev(net);
  if (rc) return rc;
  net->t += 1;
  const double c1 = 1.0 / (1.0 - std::pow((double)beta1, (double)net->t));
  const double c2 = 1.0 / (1.0 - std::pow((double)beta2, (double)net->t));
  MG_HIP(cnn::launch_adam(net->p, net->g, net->m, net->v, net->n, lr, beta1, beta2, eps, (float)c1, (float)c2,
                          net->stream));
  return prep_weights(net);
}

int magpie_cnn_sync(magpie_cnn* net) {
  if (!net) return fail(MAGPIE_ERR_INVALID_ARG, "NULL network");
  int rc = cnn_dev(net);
  if (rc) return rc;
  MG_HIP(hipStreamSynchronize(net->stream));
  return MAGPIE_OK;
}

int magpie_input_map(magpie_ctx* c, int side, float* out, int on_device) {
  if (!c || !out) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  int rc = set_dev(c);
  if (rc) return rc;
  rc = input_map_dev(c, side);
  if (rc) return rc;
  return copy_out(out, c->lrn_map, 4 * (size_t)side * side * sizeof(float), on_device, c->stream);
}

int magpie_set_object_from_coarse(magpie_ctx* c, const void* coarse, int side, int format, int on_device) {
  if (!c || !coarse) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  if (format != MAGPIE_COARSE_C64 && format != MAGPIE_COARSE_C128 && format != MAGPIE_COARSE_LOGPOLAR)
    return fail(MAGPIE_ERR_INVALID_ARG, "bad coarse format");
  if (c->nr != c->nc) return fail(MAGPIE_ERR_UNSUPPORTED, "coarse starts need a square object");
  if (side < 1 || c->nr % side || !pow2(c->nr / side))
    return fail(MAGPIE_ERR_INVALID_ARG, "object side / coarse side must be a power of two");
  int rc = set_dev(c);
  if (rc) return rc;
  const size_t bytes = (size_t)side * side *
                       (format == MAGPIE_COARSE_C64 ? sizeof(float2)
                                                     : format == MAGPIE_COARSE_C128 ? sizeof(double2) : 2 * sizeof(float));
  const void* src = coarse;
  char* tmp = nullptr;
  if (!on_device) {
    rc = dev_alloc(&tmp, bytes);
    if (rc) return rc;
    if (hipMemcpyAsync(tmp, coarse, bytes, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
      dev_free(tmp);
      return fail(MAGPIE_ERR_HIP, "coarse object upload failed");
    }
    src = tmp;
  }
  rc = prolong_into_object(c, src, side, format);
  if (!rc) rc = check_object_finite(c);   // synchronises, so tmp may be freed
  dev_free(tmp);
  return rc;
}

int magpie_restrict_object(const void* z, int n_rows, int n_cols, int times, void* out, void* stream) {
  if (!z || !out) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  if (times < 0 || times > 20) return fail(MAGPIE_ERR_INVALID_ARG, "times must be in [0, 20]");
  const int f = 1 << times;
  if (n_rows < f || n_cols < f || n_rows % f || n_cols % f)
    return fail(MAGPIE_ERR_INVALID_ARG, "2^times must divide the object's rows and columns");
  MG_HIP(cnn::launch_restrict_object((const float2*)z, n_rows, n_cols, f, (float2*)out, (hipStream_t)stream));
  return MAGPIE_OK;
}

int magpie_learned_start(magpie_ctx* c, magpie_cnn* net, double* phi_learned, double* phi_flat, int* used) {
  if (!c || !net) return fail(MAGPIE_ERR_INVALID_ARG, "NULL argument");
  if (net->device != c->device) return fail(MAGPIE_ERR_INVALID_ARG, "network and context on different devices");
  const int S = net->side, S2 = 2 * S;
  if (c->nr != c->nc || c->nr % S2 || !pow2(c->nr / S2))
    return fail(MAGPIE_ERR_INVALID_ARG, "object side / (2 * network side) must be a power of two");
  int rc = set_dev(c);
  if (rc) return rc;
  rc = input_map_dev(c, S);
  if (rc) return rc;
  MG_HIP(hipStreamSynchronize(c->stream));
  // the network reads the map's first in_ch channels (1, 3 or all 4)
  rc = magpie_cnn_forward(net, c->lrn_map, nullptr, 1, 1);
  if (rc) return rc;
  MG_HIP(hipStreamSynchronize(net->stream));
  MG_HIP(hipSetDevice(c->device));
  double pl = INFINITY, pf = 0.0;
  rc = prolong_into_object(c, net->y, S2, MAGPIE_COARSE_LOGPOLAR);
  if (rc) return rc;
  rc = magpie_objective(c, &pl, nullptr);
  if (rc == MAGPIE_ERR_NUMERIC) {
    pl = INFINITY;
  } else if (rc) {
    return rc;
  }
  if (!c->lrn_one) {
    rc = dev_alloc(&c->lrn_one, 1);
    if (rc) return rc;
    const float2 one = make_float2(1.0f, 0.0f);
    MG_HIP(hipMemcpyAsync(c->lrn_one, &one, sizeof(float2), hipMemcpyHostToDevice, c->stream));
    MG_HIP(hipStreamSynchronize(c->stream));
  }
  MG_HIP(cnn::launch_prolong_object(c->lrn_one, MAGPIE_COARSE_C64, 1, 1, c->nr, c->z, c->nr, c->nc, c->stream));
  rc = magpie_objective(c, &pf, nullptr);
  if (rc) return rc;
  const bool keep = pl < pf;
  if (keep) {
    rc = prolong_into_object(c, net->y, S2, MAGPIE_COARSE_LOGPOLAR);
    if (rc) return rc;
    MG_HIP(hipStreamSynchronize(c->stream));
  }
  if (phi_learned) *phi_learned = pl;
  if (phi_flat) *phi_flat = pf;
  if (used) *used = keep ? 1 : 0;
  return MAGPIE_OK;
}

}  // extern "C"
