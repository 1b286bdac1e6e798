// Staging of mixed table rows in LDS, shared by the matrix-core forward
// kernel and the adjoint kernel (workgroups of four waves, 64 columns).
#pragma once
#include "trx_internal.h"

namespace trx {
namespace stage {

constexpr int kWaves = 4;
constexpr int kCols = 64;

// rows[u][lane] = sum_i chi[i] * tab[i][ids[u]][col] for the corners
// u = wave, wave + NW, ... < nU of a table laid out [i][corner][W].  Loads
// are buffer loads: one resource per absorber i (its range bounds every
// access), the column as the per-lane offset and the corner row as a uniform
// offset.  A batch of kSG corners x up to kSA absorbers is issued before the
// first use and reduced per corner.
constexpr int kSG = 8;
constexpr int kSA = 4;
constexpr int kRsrcWord3 = 0x00020000;   // raw 32-bit buffer, gfx9 family
template <int NW = kWaves>
__device__ inline void stage_rows(const float* tab, int64_t abs_stride, int W, int col, const int32_t* ids,
                                  int nU, const float* chi, int nabs, float* rows, int wave, int lane) {
  const int voff = col * 4;
  const int rec = (int)(abs_stride * 4 < 0x7fffffff ? abs_stride * 4 : 0x7fffffff);
  for (int u0 = wave; u0 < nU; u0 += NW * kSG) {
    int soff[kSG];
#pragma unroll
    for (int g = 0; g < kSG; ++g) {
      const int u = u0 + NW * g < nU ? u0 + NW * g : u0;
      soff[g] = __builtin_amdgcn_readfirstlane(ids[u]) * W * 4;
    }
    float s[kSG];
#pragma unroll
    for (int g = 0; g < kSG; ++g) s[g] = 0.f;
    for (int i0 = 0; i0 < nabs; i0 += kSA) {
      float v[kSA][kSG];
#pragma unroll
      for (int ii = 0; ii < kSA; ++ii) {
        if (i0 + ii < nabs) {
          const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
              (void*)(tab + (int64_t)(i0 + ii) * abs_stride), (short)0, rec, kRsrcWord3);
#pragma unroll
          for (int g = 0; g < kSG; ++g)
            v[ii][g] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff[g], 0));
        }
      }
#pragma unroll
      for (int ii = 0; ii < kSA; ++ii) {
        if (i0 + ii < nabs) {
          const float c = __uint_as_float(__builtin_amdgcn_readfirstlane(__float_as_uint(chi[i0 + ii])));
#pragma unroll
          for (int g = 0; g < kSG; ++g) s[g] = fmaf(c, v[ii][g], s[g]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < kSG; ++g)
      if (u0 + NW * g < nU) rows[(u0 + NW * g) * kCols + lane] = s[g];
  }
}


}  // namespace stage
}  // namespace trx
