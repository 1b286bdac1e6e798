// FP64 forward kernel (the reference path): opacity (a4), optical depth
// (a5) and depth (a6) of one (model, 64-column span) per workgroup of four
// waves, with the same structure as the matrix-core kernel of the fast modes
// but FP64 throughout.
//
// The model's distinct (T, log10 P) corners are mixed over the absorbers,
// M_q = sum_i chi_i sigma_i[q], for the workgroup's 64 columns and staged in
// LDS (per 16-layer block when there are too many); so are the CIA sums.  Per
// 16-layer block each wave computes 4 layers of
//   kappa_l = sum_q w_lq M_q + w_R R + w_c0 C_0 + w_c1 C_1
// (equations opt_dpth, cia_opt_dpth, contrib; Opacities section) into LDS,
// and the optical depth tau[ray, col] += dl[ray, block] kappa[block, col] is
// accumulated on the FP64 matrix instruction v_mfma_f64_16x16x4_f64 with
// 16-ray x 16-column tiles: wave w owns the 16-ray blocks w, w+4, ... (all
// four column blocks), a ray block takes the layers at or above its first
// ray.  Models above 256 layers take several passes over the ray blocks.
// Depth: D = (Rp/Rs)^2 + sum_j (A_j/Rs^2)(-expm1(-tau_j)), the per-ray-block
// partials summed in a fixed order.
#include "trx_internal.h"

namespace trx {

namespace {

constexpr int kWaves = 4;
constexpr int kCols = 64;
constexpr int kRows = 96;                 // staged corner + CIA rows
static_assert(kRows >= kMaxU + kMaxV, "block staging must fit");
constexpr int kRBW = 4;                   // 16-ray blocks per wave per pass

typedef double f64x4 __attribute__((ext_vector_type(4)));

struct Smem64 {
  double rows[kRows][kCols];
  double kap[16][kCols];
  double part[kWaves * kRBW][kCols];
  double atm[kCols];
  double lw[16][8];
  int2 sl[16];
  int32_t ids[kRows];
  int32_t tids[kRows];
};

// rows[u][lane] = sum_i chi[i] * tab[i][ids[u]][col] (FP64 table laid out
// [i][corner][W]), corners u = wave, wave + 4, ...; 8 corners' loads of one
// absorber are issued together.
__device__ inline void stage64(const double* tab, int64_t abs_stride, int W, int col, const int32_t* ids, int nU,
                               const double* chi, int nabs, double* rows, int wave, int lane) {
  constexpr int G = 8;
  for (int u0 = wave; u0 < nU; u0 += kWaves * G) {
    int64_t off[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int u = u0 + kWaves * g < nU ? u0 + kWaves * g : u0;
      off[g] = (int64_t)__builtin_amdgcn_readfirstlane(ids[u]) * W + col;
    }
    double s[G];
#pragma unroll
    for (int g = 0; g < G; ++g) s[g] = 0.0;
    for (int i = 0; i < nabs; ++i) {
      const double* p = tab + (int64_t)i * abs_stride;
      double v[G];
#pragma unroll
      for (int g = 0; g < G; ++g) v[g] = p[off[g]];
      const double c = chi[i];
#pragma unroll
      for (int g = 0; g < G; ++g) s[g] = fma(c, v[g], s[g]);
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (u0 + kWaves * g < nU) rows[(u0 + kWaves * g) * kCols + lane] = s[g];
  }
}

__device__ void process64(const FwdArgs& a, int b_in, int span_in, Smem64& sm) {
  const int b = __builtin_amdgcn_readfirstlane(b_in);
  const int span = __builtin_amdgcn_readfirstlane(span_in);
  const Layout& L = a.L;
  const uint8_t* slab = a.ws + (int64_t)b * L.slab;
  const ModelHdr* hd = reinterpret_cast<const ModelHdr*>(slab);
  const int N = hd->n;
  if (N == 0) return;
  const int lo = hd->lo, hi = hd->hi;
  const int col0 = span * kCols;
  if (col0 >= hi || col0 + kCols <= lo) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int tid = threadIdx.x;
  const int col = col0 + lane;
  const bool valid = col >= lo && col < hi;
  const int cc = valid ? col : lo;
  const DevTables& tb = a.tab;
  const int W = tb.n_wn;
  const bool has_cia = tb.n_cia > 0;

  double R = 0.0;
  if (tb.has_rayleigh)
    for (int s = 0; s < tb.n_abs + 2; ++s) R = fma(hd->chi_s[s], tb.ray64[(int64_t)s * W + cc], R);

  const double* lw = reinterpret_cast<const double*>(slab + L.off_lw64);
  const int32_t* lid = reinterpret_cast<const int32_t*>(slab + L.off_lid);
  const KBlk* kblk = reinterpret_cast<const KBlk*>(slab + L.off_kblk);
  const MList* ml = reinterpret_cast<const MList*>(slab + L.off_mlist);
  const double* A = reinterpret_cast<const double*>(slab + L.off_A64);
  const double* dlT = reinterpret_cast<const double*>(slab + L.off_dl);
  const int NP = L.NP;
  const int nkb = (N + 15) / 16;
  const int64_t abs_stride = (int64_t)tb.n_T * tb.n_P * W;
  const int64_t cia_stride = (int64_t)tb.n_Tcia * W;

  double* rows = &sm.rows[0][0];
  double* crows = rows;
  auto stage = [&](const int32_t* ids, int nU, const int32_t* tids, int nV) {
    for (int e = tid; e < nU; e += 64 * kWaves) sm.ids[e] = ids[e];
    for (int e = tid; e < nV; e += 64 * kWaves) sm.tids[e] = tids[e];
    __syncthreads();
    stage64(tb.xsec64, abs_stride, W, cc, sm.ids, nU, hd->chi_s, tb.n_abs, rows, wave, lane);
    crows = rows + nU * kCols;
    if (has_cia) stage64(tb.cia64, cia_stride, W, cc, sm.tids, nV, hd->cia_w, tb.n_cia, crows, wave, lane);
  };
  const bool mstage = ml->nU + ml->nV <= kRows && ml->nV <= kMListV;
  const int slot_off = mstage ? 2 : 4;
  if (mstage) stage(ml->ids, ml->nU, ml->tids, ml->nV);
  if (tid < kCols) sm.atm[tid] = 0.0;

  const int nrb16 = (N + 15) / 16;
  for (int p0 = 0; p0 < nrb16; p0 += kWaves * kRBW) {
    f64x4 acc[kRBW][4];
#pragma unroll
    for (int r = 0; r < kRBW; ++r)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[r][cb] = f64x4{0.0, 0.0, 0.0, 0.0};
    // ray block p0 starts at ray 16 p0: layer blocks from p0 on
    for (int kb = p0; kb < nkb; ++kb) {
      if (!mstage) {
        const KBlk* kd = kblk + kb;
        stage(kd->ids, kd->nU, kd->tids, kd->nV);
      }
      if (tid < 16 * 8) {
        const int l = 16 * kb + tid / 8;
        sm.lw[tid / 8][tid % 8] = l < N ? lw[8 * l + tid % 8] : 0.0;
      }
      if (tid < 16) {
        const int l = 16 * kb + tid;
        sm.sl[tid] = l < N ? *reinterpret_cast<const int2*>(lid + 8 * l + slot_off) : make_int2(0, 0);
      }
      __syncthreads();
      // opacity of layers 16 kb + 4 wave + jj
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int k = 4 * wave + jj;
        const int l = 16 * kb + k;
        double kv = 0.0;
        if (l < N) {
          const double* w = sm.lw[k];
          const uint32_t sl = __builtin_amdgcn_readfirstlane((uint32_t)sm.sl[k].x);
          kv = w[0] * rows[(sl & 0xff) * kCols + lane];
          kv = fma(w[1], rows[((sl >> 8) & 0xff) * kCols + lane], kv);
          kv = fma(w[2], rows[((sl >> 16) & 0xff) * kCols + lane], kv);
          kv = fma(w[3], rows[(sl >> 24) * kCols + lane], kv);
          kv = fma(w[4], R, kv);
          if (has_cia) {
            const uint32_t cl = __builtin_amdgcn_readfirstlane((uint32_t)sm.sl[k].y);
            kv = fma(w[5], crows[(cl & 0xff) * kCols + lane], kv);
            kv = fma(w[6], crows[((cl >> 8) & 0xff) * kCols + lane], kv);
          }
        }
        sm.kap[k][lane] = kv;
      }
      __syncthreads();
      // tau += dl x kappa on 16x16x4 FP64 tiles; A operand lane l holds
      // dl[16 rb + l%16][4 s + l/16], B operand kappa[4 s + l/16][16 cb + l%16]
#pragma unroll
      for (int r = 0; r < kRBW; ++r) {
        const int rb = p0 + wave + kWaves * r;
        if (rb < nrb16 && kb >= rb) {
#pragma unroll
          for (int st = 0; st < 4; ++st) {
            const int k = 4 * st + (lane >> 4);
            const double av = dlT[(int64_t)(16 * kb + k) * NP + 16 * rb + (lane & 15)];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
              const double bv = sm.kap[k][16 * cb + (lane & 15)];
              acc[r][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[r][cb], 0, 0, 0);
            }
          }
        }
      }
      __syncthreads();
    }
    // depth partials: accumulator element q of lane l is ray l/16 + 4 q of
    // the block (the FP64 instruction interleaves its output rows)
#pragma unroll
    for (int r = 0; r < kRBW; ++r) {
      const int rb = p0 + wave + kWaves * r;
      if (rb < nrb16) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          double s = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int j = 16 * rb + (lane >> 4) + 4 * q;
            s = fma(A[j], -expm1(-acc[r][cb][q]), s);
          }
          s += __shfl_xor(s, 16, 64);
          s += __shfl_xor(s, 32, 64);
          if (lane < 16) sm.part[wave + kWaves * r][16 * cb + lane] = s;
        }
      } else if (lane < 16) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) sm.part[wave + kWaves * r][16 * cb + lane] = 0.0;
      }
    }
    __syncthreads();
    if (tid < kCols) {
      // slot wave + 4 r holds ray block p0 + wave + 4 r: summed in ray order
      double s = sm.atm[tid];
      for (int i = 0; i < kWaves * kRBW; ++i) s += sm.part[i][tid];
      sm.atm[tid] = s;
    }
    __syncthreads();
  }
  if (tid < kCols && valid) {
    const double atm = sm.atm[tid];
    const int64_t o = (int64_t)b * W + col;
    reinterpret_cast<double*>(a.aws)[o] = atm;
    if (a.depth_native) a.depth_native[o] = hd->Rp2_Rs2 + atm;
    if (!isfinite(atm)) atomicOr(&a.model_status[b], TRX_MODEL_NONFINITE);
  }
  __syncthreads();
}

__global__ __launch_bounds__(64 * kWaves) void k_fwd64(FwdArgs a) {
  __shared__ Smem64 sm;
  const int B = a.B_dev ? *a.B_dev : a.B;
  if ((int)blockIdx.x >= B) return;
  process64(a, blockIdx.x, blockIdx.y, sm);
}

}  // namespace

void launch_fwd64(const FwdArgs& a, int B_grid, hipStream_t s) {
  if (B_grid <= 0) return;
  const int spans = (a.tab.n_wn + kCols - 1) / kCols;
  hipLaunchKernelGGL(k_fwd64, dim3(B_grid, spans), dim3(64 * kWaves), 0, s, a);
}

}  // namespace trx
