// Matrix-core forward kernel for the FP32 and split-bf16 modes: opacity
// (a4), optical depth (a5) and depth (a6) of one (model, 256-column span)
// per workgroup, one 64-column slice per wave.
//
// Opacity.  Each lane owns one wavenumber column and computes the absorption
// coefficient of the 16 layers of a layer block in FP32 from the
// mixing-ratio-weighted corner values of the layer's (T, log10 P) bracket
// (equations opt_dpth, cia_opt_dpth, contrib; Opacities section), exactly as
// in the FP64 kernel but in FP32 from the FP32 tables.
//
// Optical depth.  tau[ray, col] = sum_k dl[ray, k] kappa[k, col] is the
// matrix product dl (rays x layers, upper triangular) x kappa (layers x
// columns), done on the matrix cores with 32x32 output tiles: a wave holds
// the accumulators of every 32-ray block for its two 32-column blocks and
// walks the layer blocks once; a ray block only takes layer blocks at or
// above its first ray (the triangle).  The opacity block computed by a lane
// (one column, 16 layers) is turned into the B operand layout with one
// v_permlane32_swap per register pair (lanes l and l+32 exchange halves).
//   FP32 mode: v_mfma_f32_32x32x2_f32 with kappa in FP32 and the path
//     lengths in two FP32 pieces (hi + lo), two products.
//   bf16 modes: v_mfma_f32_32x32x16_bf16 with both operands split into bf16
//     pieces, x = x0 + x1 (+ x2); the products x0*y0 + x0*y1 + x1*y0 (two
//     pieces) or all products with piece-index sum <= 2 (three pieces) are
//     accumulated in FP32, recovering ~16 or ~24 bits of the operands.
//
// Depth.  Each accumulator element is a (ray, column) optical depth; the
// lane adds (A_j/Rs^2)(1 - exp(-tau)) over its 16 rows per ray block and the
// two lanes sharing a column combine with one cross-lane exchange.
#include "trx_internal.h"

namespace trx {

namespace {

constexpr int kWaves = 4;
constexpr int kSpan = 64 * kWaves;

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct Mixer32 {
  const float* xs;
  const float* ci;
  int64_t abs_stride, cia_stride;
  int W, nP, nabs, ncia;
  const float* chi;
  const float* ciaw;

  __device__ float corner(int c) const {
    float s = 0.f;
    const float* p = xs + (int64_t)c * W;
    for (int i = 0; i < nabs; ++i) s = fmaf(chi[i], p[i * abs_stride], s);
    return s;
  }
  __device__ float cia(int t) const {
    float s = 0.f;
    const float* p = ci + (int64_t)t * W;
    for (int q = 0; q < ncia; ++q) s = fmaf(ciaw[q], p[q * cia_stride], s);
    return s;
  }
};

struct Corners32 {
  int base = -1 << 30, cbase = -1 << 30;
  float c00 = 0, c10 = 0, c01 = 0, c11 = 0, C0 = 0, C1 = 0;

  __device__ void update(const Mixer32& m, int nb, int ncb) {
    const int nP = m.nP;
    if (nb != base) {
      if (nb == base - 1) {
        c01 = c00; c11 = c10;
        c00 = m.corner(nb); c10 = m.corner(nb + nP);
      } else if (nb == base + 1) {
        c00 = c01; c10 = c11;
        c01 = m.corner(nb + 1); c11 = m.corner(nb + nP + 1);
      } else if (nb == base + nP) {
        c00 = c10; c01 = c11;
        c10 = m.corner(nb + nP); c11 = m.corner(nb + nP + 1);
      } else if (nb == base - nP) {
        c10 = c00; c11 = c01;
        c00 = m.corner(nb); c01 = m.corner(nb + 1);
      } else {
        c00 = m.corner(nb); c10 = m.corner(nb + nP);
        c01 = m.corner(nb + 1); c11 = m.corner(nb + nP + 1);
      }
      base = nb;
    }
    if (m.ncia > 0 && ncb != cbase) {
      if (ncb == cbase + 1) { C0 = C1; C1 = m.cia(ncb + 1); }
      else if (ncb == cbase - 1) { C1 = C0; C0 = m.cia(ncb); }
      else { C0 = m.cia(ncb); C1 = m.cia(ncb + 1); }
      cbase = ncb;
    }
  }
};

__device__ inline uint32_t swap_lo(uint32_t x, uint32_t y, uint32_t& hi_out) {
  // v_permlane32_swap: the upper 32 lanes of x trade places with the lower
  // 32 lanes of y.  Returns the new x; the new y goes to hi_out.
  auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
  hi_out = r[1];
  return r[0];
}

__device__ inline uint32_t bf16_pair(float a, float b) {
  __bf16 ha = (__bf16)a, hb = (__bf16)b;
  return (uint32_t)__builtin_bit_cast(uint16_t, ha) | ((uint32_t)__builtin_bit_cast(uint16_t, hb) << 16);
}
__device__ inline float bf16_lo_f(uint32_t p) { return __uint_as_float(p << 16); }
__device__ inline float bf16_hi_f(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }

template <int MODE>
struct Pieces {
  static constexpr int n = MODE == TRX_BF16_SPLIT3 ? 3 : 2;
};

template <int MODE, int NRB>
__global__ __launch_bounds__(64 * kWaves) void k_fwd_mfma(FwdArgs a) {
  const int b = blockIdx.x;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if (b >= B) return;
  const Layout& L = a.L;
  const uint8_t* slab = a.ws + (int64_t)b * L.slab;
  const ModelHdr* h = reinterpret_cast<const ModelHdr*>(slab);
  const int N = h->n;
  if (N == 0) return;
  const int lo = h->lo, hi = h->hi;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col0 = blockIdx.y * kSpan + wave * 64;
  if (col0 >= hi || col0 + 64 <= lo) return;
  const int col = col0 + lane;
  const bool valid = col >= lo && col < hi;
  const int cc = valid ? col : lo;
  const DevTables& tb = a.tab;
  const int W = tb.n_wn;

  Mixer32 m;
  m.xs = tb.xsec32 + cc;
  m.ci = tb.cia32 + cc;
  m.abs_stride = (int64_t)tb.n_T * tb.n_P * W;
  m.cia_stride = (int64_t)tb.n_Tcia * W;
  m.W = W; m.nP = tb.n_P; m.nabs = tb.n_abs; m.ncia = tb.n_cia;
  m.chi = h->chi_s32;
  m.ciaw = h->cia_w32;

  float R = 0.f;
  if (tb.has_rayleigh)
    for (int s = 0; s < tb.n_abs + 2; ++s) R = fmaf(h->chi_s32[s], tb.ray32[(int64_t)s * W + cc], R);

  const float* lw = reinterpret_cast<const float*>(slab + L.off_lw32);
  const int32_t* lid = reinterpret_cast<const int32_t*>(slab + L.off_lid);
  const float* Aw = reinterpret_cast<const float*>(slab + L.off_A32);
  const uint8_t* frag = slab + L.off_dl;
  const int nkb = h->nkb, nrb = h->nrb;
  const int NKB = L.NKB;

  f32x16 acc[NRB][2];
#pragma unroll
  for (int r = 0; r < NRB; ++r) {
    acc[r][0] = f32x16{};
    acc[r][1] = f32x16{};
  }
  Corners32 cs;
  const int hl = lane >> 5;

  for (int kb = 0; kb < nkb; ++kb) {
    float kap[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int l = 16 * kb + j;
      if (l < N) {
        cs.update(m, lid[2 * l], lid[2 * l + 1]);
        const float* w = lw + 8 * l;
        float k = w[0] * cs.c00;
        k = fmaf(w[1], cs.c10, k);
        k = fmaf(w[2], cs.c01, k);
        k = fmaf(w[3], cs.c11, k);
        k = fmaf(w[4], R, k);
        k = fmaf(w[5], cs.C0, k);
        k = fmaf(w[6], cs.C1, k);
        kap[j] = k;
      } else {
        kap[j] = 0.f;
      }
    }
    if constexpr (MODE == TRX_FP32) {
      // B operand of 32x32x2, step i: lane l holds kappa[2i + l/32][col l%32].
      uint32_t b0[8], b1[8];
#pragma unroll
      for (int i = 0; i < 8; ++i)
        b0[i] = swap_lo(__float_as_uint(kap[2 * i]), __float_as_uint(kap[2 * i + 1]), b1[i]);
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) {
        if (rb < nrb && kb >= 2 * rb) {
          const float* fp = reinterpret_cast<const float*>(frag) +
                            (int64_t)frag_index(rb, kb, NKB) * 2 * 512 + lane * 8;
          const float4 h0 = *reinterpret_cast<const float4*>(fp);
          const float4 h1 = *reinterpret_cast<const float4*>(fp + 4);
          const float4 l0 = *reinterpret_cast<const float4*>(fp + 512);
          const float4 l1 = *reinterpret_cast<const float4*>(fp + 516);
          const float ah[8] = {h0.x, h0.y, h0.z, h0.w, h1.x, h1.y, h1.z, h1.w};
          const float al[8] = {l0.x, l0.y, l0.z, l0.w, l1.x, l1.y, l1.z, l1.w};
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const float x0 = __uint_as_float(b0[i]), x1 = __uint_as_float(b1[i]);
            acc[rb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ah[i], x0, acc[rb][0], 0, 0, 0);
            acc[rb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(al[i], x0, acc[rb][0], 0, 0, 0);
            acc[rb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ah[i], x1, acc[rb][1], 0, 0, 0);
            acc[rb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(al[i], x1, acc[rb][1], 0, 0, 0);
          }
        }
      }
    } else {
      constexpr int NPC = Pieces<MODE>::n;
      // split kappa into bf16 pieces, packed by layer pairs (2d, 2d+1)
      uint32_t pk[NPC][8];
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        float x0 = kap[2 * d], x1 = kap[2 * d + 1];
#pragma unroll
        for (int p = 0; p < NPC; ++p) {
          const uint32_t q = bf16_pair(x0, x1);
          pk[p][d] = q;
          x0 -= bf16_lo_f(q);
          x1 -= bf16_hi_f(q);
        }
      }
      // B operand of 32x32x16: lane l holds kappa[8 (l/32) + v][col l%32];
      // column block 0 = columns 0..31 of the wave, block 1 = 32..63.
      u32x4 B0[NPC], B1[NPC];
#pragma unroll
      for (int p = 0; p < NPC; ++p) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          uint32_t y;
          B0[p][d] = swap_lo(pk[p][d], pk[p][d + 4], y);
          B1[p][d] = y;
        }
      }
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb) {
        if (rb < nrb && kb >= 2 * rb) {
          const u32x4* fp = reinterpret_cast<const u32x4*>(frag + ((int64_t)frag_index(rb, kb, NKB) * NPC * 512 +
                                                                  lane * 8) * 2);
          u32x4 Ap[NPC];
#pragma unroll
          for (int p = 0; p < NPC; ++p) Ap[p] = fp[p * 64];
#pragma unroll
          for (int pa = 0; pa < NPC; ++pa) {
#pragma unroll
            for (int pb = 0; pb + pa < NPC; ++pb) {
              const bf16x8 av = __builtin_bit_cast(bf16x8, Ap[pa]);
              acc[rb][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  av, __builtin_bit_cast(bf16x8, B0[pb]), acc[rb][0], 0, 0, 0);
              acc[rb][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  av, __builtin_bit_cast(bf16x8, B1[pb]), acc[rb][1], 0, 0, 0);
            }
          }
        }
      }
    }
  }

  // depth: rows of accumulator register r are 8 (r/4) + 4 (l/32) + r%4
  float s0 = 0.f, s1 = 0.f;
  const float nl2e = -1.4426950408889634f;
#pragma unroll
  for (int rb = 0; rb < NRB; ++rb) {
    if (rb < nrb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * rb + 8 * (r >> 2) + 4 * hl + (r & 3);
        const float A = Aw[row];
        s0 = fmaf(A, 1.f - exp2f(nl2e * acc[rb][0][r]), s0);
        s1 = fmaf(A, 1.f - exp2f(nl2e * acc[rb][1][r]), s1);
      }
    }
  }
  s0 += __shfl_xor(s0, 32, 64);
  s1 += __shfl_xor(s1, 32, 64);
  if (valid) {
    const float atm = hl ? s1 : s0;
    const int64_t o = (int64_t)b * W + col;
    reinterpret_cast<float*>(a.aws)[o] = atm;
    if (a.depth_native) a.depth_native[o] = h->Rp2_Rs2 + (double)atm;
    if (!isfinite(atm)) atomicOr(&a.model_status[b], TRX_MODEL_NONFINITE);
  }
}

template <int MODE>
void launch_mode(const FwdArgs& a, int nrb, int B_grid, hipStream_t s) {
  dim3 grid(B_grid, a.n_spans), blk(64 * kWaves);
  if (nrb <= 2) hipLaunchKernelGGL((k_fwd_mfma<MODE, 2>), grid, blk, 0, s, a);
  else if (nrb <= 4) hipLaunchKernelGGL((k_fwd_mfma<MODE, 4>), grid, blk, 0, s, a);
  else hipLaunchKernelGGL((k_fwd_mfma<MODE, 7>), grid, blk, 0, s, a);
}

}  // namespace

void launch_fwd_mfma(const FwdArgs& a, int precision, int nrb_max, int B_grid, int persistent_grid,
                     hipStream_t s) {
  (void)persistent_grid;
  if (B_grid <= 0 || a.n_spans <= 0) return;
  switch (precision) {
    case TRX_FP32: launch_mode<TRX_FP32>(a, nrb_max, B_grid, s); break;
    case TRX_BF16_SPLIT2: launch_mode<TRX_BF16_SPLIT2>(a, nrb_max, B_grid, s); break;
    default: launch_mode<TRX_BF16_SPLIT3>(a, nrb_max, B_grid, s); break;
  }
}

}  // namespace trx
