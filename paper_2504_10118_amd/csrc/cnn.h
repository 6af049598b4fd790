// Launch interface of the learned-start kernels (cnn.hip): 3x3 convolutions
// and their gradients, the complex MSE head, Adam, the network input map built
// from measured intensities, and whole-object restriction / prolongation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cnn {

constexpr int CONV_TILE = 16;        // output pixels per workgroup side
constexpr int MAX_WIDTH = 32;        // channels handled by one thread (wgrad: 4 output x 32 input channels)

// out = conv3x3(in) with zero padding 1.  in: [B][ci][Hi][Wi] (Hi = H/2 when up,
// read through nearest 2x upsampling), w: [co][ci][9] float or bf16 bits,
// out: [B][co][H][W].  mode 0: + bias, ReLU; 1: + bias; 2: no bias, zero where
// omask <= 0 (omask has out's shape); 3: no bias.
hipError_t launch_conv(int co, bool up, int mode, bool bf16, const float* in, const void* w, const float* bias,
                       float* out, const float* omask, int batch, int ci, int H, int W, hipStream_t s);

// Per-workgroup partial weight and bias gradients of a 3x3 convolution:
// part[wg][(co*ci + c)*9 + t] and part[wg][co*ci*9 + co]; wgrad_workgroups
// gives the number of workgroups (rows of part).  in holds the convolution's
// input (read through upsampling when up), dout its output gradient
// [B][co][H][W].
int wgrad_workgroups(int batch, int H, int W);
constexpr int WGRAD_MAX_WORKGROUPS = 512;   // upper bound of wgrad_workgroups for any shape
hipError_t launch_wgrad(bool up, const float* in, const float* dout, float* part, int batch, int ci, int co, int H,
                        int W, hipStream_t s);
// grad[j] = sum over rows of part (fixed order), j < row_len.
hipError_t launch_rows_sum(const float* part, int n_rows, int row_len, float* grad, hipStream_t s);

// da[b][c][y][x] = (a > 0) ? sum of du over the 2x2 block : 0 (adjoint of the
// upsampling followed by the ReLU mask).  da, a: [B][C][H][W]; du: [B][C][2H][2W].
hipError_t launch_up_backward_mask(const float* du, const float* a, float* da, int batch, int C, int H, int W,
                                   hipStream_t s);

// Masked complex MSE of exp(y0 + i y1) against target; dy gets the gradient.
// y, dy: [B][2][HW]; target: [B][HW] complex; mask: [HW].  Per-block FP64 loss
// partials go to part (n_blocks returned by cmse_blocks).  With rot non-null
// each sample's prediction is first rotated by its best global phase
// (rot[b] = ip / |ip|, ip = sum mask conj(pred) t, partials in ip_part
// [B][cmse_ip_blocks(hw)]).
int cmse_blocks(int batch, int hw);
int cmse_ip_blocks(int hw);
hipError_t launch_cmse(const float* y, const float2* target, const float* mask, float2* rot, double2* ip_part,
                       float* dy, double* part, int batch, int hw, float inv_norm, hipStream_t s);
hipError_t launch_sum_f64(const double* x, int n, double* out, hipStream_t s);

// Adam with bias corrections c1 = 1/(1-b1^t), c2 = 1/(1-b2^t).
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);

// Compute copies of a layer's weights: wf[co][ci][t] and the transposed,
// flipped wt[ci][co][8 - t] (the backward-data convolution), float or bf16.
hipError_t launch_prep_weights(const float* p, void* wf, void* wt, int co, int ci, bool bf16, hipStream_t s);

// Network input map.  stats[k] = (mean sqrt(d_k) * qinv, row and column
// frequency centres of mass of d_k, 0) from sqrt(d) in natural order.
hipError_t launch_probe_norm(const double2* q, int m, double* out, hipStream_t s);
hipError_t launch_position_stats(const float* sqrtd, int n_pos, int m, const double* qnorm, double4* stats,
                                 hipStream_t s);
// fine[ch][r][c] = sum_k |Q(p-o_k)|^2 stats[k][ch] / sum_k |Q(p-o_k)|^2 over the positions
// in the pixel's tile list (0 where uncovered), ch < 3.
hipError_t launch_map_fine(const double4* stats, const double2* q, int m, const int* tile_ptr, const int4* tile_ent,
                           int tiles_x, int tile_w, int tile_h, int nr, int nc, double* fine, hipStream_t s);
// out[ch][i][j] = mean of fine[ch] over the fr x fc block (i, j).
hipError_t launch_pool(const double* fine, int nr, int nc, int fr, int fc, float* out, hipStream_t s);
// out = the S x S phase whose gradient is (sy * gy, sx * gx) in the least-squares
// (periodic, spectral) sense, mean 0; S <= 64.
constexpr int PHASE_MAX_SIDE = 64;
hipError_t launch_integrate_phase(const float* gy, const float* gx, int S, double sy, double sx, float* out,
                                  hipStream_t s);

// z[r][c] = coarse[r / f][c / f]; format 0 complex64, 1 complex128, 2 planes
// (log-amplitude, phase) float [2][sr][sc].
hipError_t launch_prolong_object(const void* coarse, int format, int sr, int sc, int f, float2* z, int nr, int nc,
                                 hipStream_t s);
// out[i][j] = mean of z over the f x f block (i, j) (complex64 in and out).
hipError_t launch_restrict_object(const float2* z, int nr, int nc, int f, float2* out, hipStream_t s);

}  // namespace cnn
