// Binning kernel (a7): channel c of model b is the weighted mean over the
// native points i of the model's window,
//   D_c = sum_i w_ci D_i / sum_i w_ci   (Binning subsection),
// with w_ci the overlap of the native bin and the channel divided by the
// native bin width.  Since the weights are normalised, the (Rp/Rs)^2 part
// of D passes through unchanged and only the atmospheric part a_i/Rs^2 is
// averaged (in FP64).  One wave per (channel, model); the sum runs in a
// fixed order, so repeated launches give identical bits.
#include "trx_internal.h"

namespace trx {

namespace {

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(64) void k_bin(BinArgs a) {
  const int c = blockIdx.x, b = blockIdx.y;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if (b >= B) return;
  const ModelHdr* h = reinterpret_cast<const ModelHdr*>(a.ws + (int64_t)b * a.L.slab);
  const int lane = threadIdx.x;
  double* out = a.out + (int64_t)b * a.n_ch + c;
  if (h->status != 0) {
    if (lane == 0) *out = __builtin_nan("");
    return;
  }
  const int c0 = a.ch_i0[c];
  const int i0 = max(c0, h->lo), i1 = min(a.ch_i1[c], h->hi);
  const double* w = a.ch_w + a.ch_off[c] - c0;
  double sw = 0.0, swa = 0.0;
  const int64_t row = (int64_t)b * a.n_wn;
  if (a.aws_f64) {
    const double* x = reinterpret_cast<const double*>(a.aws) + row;
    for (int i = i0 + lane; i < i1; i += 64) { sw += w[i]; swa = fma(w[i], x[i], swa); }
  } else {
    const float* x = reinterpret_cast<const float*>(a.aws) + row;
    for (int i = i0 + lane; i < i1; i += 64) { sw += w[i]; swa = fma(w[i], (double)x[i], swa); }
  }
  sw = wave_sum(sw);
  swa = wave_sum(swa);
  if (lane == 0) *out = (sw > 0.0) ? h->Rp2_Rs2 + swa / sw : __builtin_nan("");
}

}  // namespace

void launch_bin(const BinArgs& a, int B_grid, hipStream_t s) {
  if (B_grid <= 0 || a.n_ch <= 0) return;
  hipLaunchKernelGGL(k_bin, dim3(a.n_ch, B_grid), dim3(64), 0, s, a);
}

}  // namespace trx
