// HIP kernels (gfx950 / CDNA4) of the SRM EM sweep, arXiv 1608.04647 Sec. II.
//
// Data layout in HBM (all row-major, zero padded):
//   Xhat   : sum_i vp_i rows x ldt columns, one plane (FP32 or BF16) or two
//            planes (BF16 hi, BF16 lo).  vp_i = round_up(v_i, 32),
//            ldt = round_up(t, 64) (128 for the one-pass sweep).  Subjects
//            are stacked; row r is global.
//   A, S   : "records", i.e. the exact per-lane operand layout of the
//            matrix-core instructions, so a wave loads an operand tile with one
//            contiguous 1-2 KiB access and never shuffles it.
//     A record (32 rows x 16 columns of A = Xhat S^T, or of W0 at start):
//            lane l holds A[32 rb + row(l/16, e)][16 jb + l%16], e = 0..7,
//            row(g, e) = 4 g + (e & 3) + 16 (e >> 2).  This is at once the
//            16x16 accumulator layout of two stacked M-phase output tiles and
//            the K = rows operand layout of the E-phase.
//     S record, BF16 forms (32 TRs x 16 features):
//            lane l holds S[16 jb + l%16][32 tb + 8 (l/16) + e], e = 0..7.
//     S record, FP32 (16 TRs x 16 features):
//            lane l holds S[16 jb + l%16][16 tb + 4 (l/16) + s], s = 0..3.
//
// Per EM iteration (deferred W: W_i = A_i P_i with P_i = (A_i^T A_i)^-1/2):
//   k_fused    one-pass sweep (BF16 forms, K padding <= 64, ldt <= 512):
//              A = Xhat S^T per chunk in LDS, then Z_s = A_s^T Xhat_s and
//              G_s = A_s^T A_s per slice (Eq. 4 numerator and Gram, Eq. 10
//              partials); A never goes to HBM
//   k_mphase   two-pass sweep, pass 1: A = Xhat S^T (Eq. 4 numerator, A_i)
//   k_ephase   two-pass sweep, pass 2: Z_s and G_s per slice from A
//   k_gram_z   sample-space variant: Z_i = S G_i and S G_i S^T from
//              G_i = Xhat_i^T Xhat_i, formed once by k_gram_build
//   k_polar    G_i -> P_i = G_i^-1/2 (FP64): Newton-Schulz from the previous
//              P_i, else cyclic Jacobi; tr(W_i^T A_i), rho_i^2 (Eq. 4-5)
//   k_ereduce  Y = sum_i rho_i^-2 P_i sum_s Z_s   (Eq. 10 reduction, FP64)
//   k_post_prep rho0, M = (Sigma_s^-1 + rho0 I)^-1, log-det (Eq. 7-8, FP64)
//   k_post_s   S = M Y (Eq. 10 with Sigma_s [I - rho0 M] = M), S S^T partials
//   k_post_sig Sigma_s = M + S S^T / t (Eq. 11)
//   k_post_fin tr(Sigma_s) (for Eq. 5), log-likelihood
// All reductions run in a fixed order: results are bitwise reproducible.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "srm_internal.h"

namespace srm {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ f32x4 mfma_bf16(uint4 a, uint4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b),
                                                 c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Round-to-nearest-even float -> bfloat16 bits (inputs are finite).
__device__ __forceinline__ uint32_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf2f(uint32_t h) {
  return __uint_as_float(h << 16);
}
// Two floats to packed bfloat16 bits (a in the low half), round to nearest
// even by the hardware conversion (v_cvt_pk_bf16_f32); equal to f2bf on
// finite inputs.
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  typedef float f32x2_t __attribute__((ext_vector_type(2)));
  const f32x2_t v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}
// hi = bf16(a, b) packed, lo = bf16(a - hi_a, b - hi_b) packed.
__device__ __forceinline__ void split2(float a, float b, uint32_t& hi, uint32_t& lo) {
  hi = pk_bf16(a, b);
  lo = pk_bf16(a - __uint_as_float(hi << 16), b - __uint_as_float(hi & 0xffff0000u));
}

// hi = bf16(v), lo = bf16(v - hi), packed 8 -> uint4 each.
__device__ __forceinline__ void split8(const float (&v)[8], uint4& hi,
                                       uint4& lo) {
  uint32_t h[8], l[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    h[e] = f2bf(v[e]);
    l[e] = f2bf(v[e] - bf2f(h[e]));
  }
  hi = make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16),
                  h[4] | (h[5] << 16), h[6] | (h[7] << 16));
  lo = make_uint4(l[0] | (l[1] << 16), l[2] | (l[3] << 16),
                  l[4] | (l[5] << 16), l[6] | (l[7] << 16));
}


// Buffer loads: a wave-uniform descriptor (base, byte size) plus a 32-bit
// per-lane offset and a scalar offset.  Keeps per-load 64-bit addresses out
// of vector registers in the streaming loops.
typedef __attribute__((ext_vector_type(4))) unsigned v4u;
typedef __attribute__((ext_vector_type(2))) unsigned v2u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           0x00020000);
}
__device__ __forceinline__ uint4 bload16(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  const v4u v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint2 bload8(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  const v2u v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  return make_uint2(v.x, v.y);
}

// LDS read with a transpose (gfx950 ds_read_b64_tr_b16): in each group of
// 16 lanes, lane 4 r + q supplies four consecutive 16-bit values that become
// positions 4 q .. 4 q + 3 of row r (r, q = 0..3), and lane i receives
// position i of rows 0..3.  p is this lane's LDS byte address.
typedef short v4s __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4s ds_tr16(const char* p) {
  return __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (__attribute__((address_space(3))) v4s*)(p));
}
// Direct load of 16 bytes per lane from a buffer into LDS: lane j's bytes
// land at lds + 16 j (lds wave-uniform).  Written as one asm statement (M0 is
// set in it) so that the compiler does not guard every later LDS read with a
// wait for all outstanding loads: the caller waits for these loads itself
// (s_waitcnt vmcnt) and then synchronises the workgroup before reading.
// M0 is reserved by the compiler, which sets it right before each of its
// own uses, so it is left off the clobber list.
typedef int v4i_rsrc __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4i_rsrc make_rsrc_v4(const void* p, uint32_t bytes) {
  const uint64_t a = (uint64_t)p;
  return v4i_rsrc{(int)(uint32_t)a, (int)(uint32_t)(a >> 32), (int)bytes, 0x00020000};
}
__device__ __forceinline__ void load_lds16(v4i_rsrc r, const void* lds, int voff, int soff) {
  const uint32_t m = __builtin_amdgcn_readfirstlane(
      (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char*)(lds));
  asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dwordx4 %1, %2, %3 offen lds"
               :: "s"(m), "v"(voff), "s"(r), "s"(soff) : "memory");
}

// A slice descriptor read through the scalar unit (the table is written
// before the launch and only read during it): row0 and nrows, wave-uniform.
// The wait sits in the same statement, so the outputs are complete when the
// statement ends.
__device__ __forceinline__ void slice_s(const Slice* p, int64_t& row0, int32_t& nrows) {
  v4i_rsrc v;
  asm volatile("s_load_dwordx4 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(v) : "s"(p));
  row0 = (int64_t)(uint32_t)v.x | ((int64_t)(uint32_t)v.y << 32);
  nrows = v.z;
}

// Two transposed reads (4 + 4 values) -> one 8-value bf16 operand.
__device__ __forceinline__ uint4 pack_tr(v4s a, v4s b) {
  const uint2 x = __builtin_bit_cast(uint2, a), y = __builtin_bit_cast(uint2, b);
  return make_uint4(x.x, x.y, y.x, y.y);
}

// Workgroup ids are dealt round-robin to the 8 XCDs; map them so that
// consecutive logical ids share an XCD (and its L2).
__device__ __forceinline__ int xcd_remap(int h, int G) {
  const int q = G >> 3, r = G & 7;
  const int x = h & 7, l = h >> 3;
  return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order block sum over 256 threads (result valid in every thread).
__device__ double block_sum256(double v, double* red /* >= 4 */) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// Sum over a workgroup of NT threads, in a fixed order.
template <int NT>
__device__ double block_sum_nt(double v, double* red /* >= NT / 64 */) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) r += red[w];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Initialisation: demean (Algorithm 1), convert, per-row ||xhat||^2.
// One wave per (padded) global row of one subject.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_convert(ConvertArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t r = a.row_begin + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= a.row_end) return;
  const int64_t lr = r - a.subj_row0;
  const bool real = lr < a.v;
  const float* src = real ? a.src + (lr - a.src_row0) * a.t : nullptr;
  double s = 0.0;
  bool bad = false;
  if (real) {
    for (int64_t c = lane; c < a.t; c += 64) {
      const float x = src[c];
      bad |= !isfinite(x);
      s += (double)x;
    }
  }
  s = wave_sum(s);
  const double mu = real ? s / (double)a.t : 0.0;
  // Optional standardisation: population standard deviation over the
  // samples.  A constant row keeps scale 1: the FP64 sum of equal float32
  // values is exact, so its mean is exact and its deviations are zero.
  double inv = 1.0;
  if (a.zscore && real) {
    double ss = 0.0;
    for (int64_t c = lane; c < a.t; c += 64) {
      const double d = (double)src[c] - mu;
      ss += d * d;
    }
    ss = wave_sum(ss);
    const double sd = sqrt(ss / (double)a.t);
    if (sd > 0.0) inv = 1.0 / sd;
  }
  double sq = 0.0;
  for (int64_t c = lane; c < a.ldt; c += 64) {
    const float f = (real && c < a.t) ? (float)(((double)src[c] - mu) * inv) : 0.0f;
    const int64_t o = r * a.ldt + c;
    if (a.prec == P_FP32) {
      ((float*)a.xh)[o] = f;
      sq += (double)f * (double)f;
    } else {
      const uint32_t h = f2bf(f);
      ((uint16_t*)a.xh)[o] = (uint16_t)h;
      double st = (double)bf2f(h);
      if (a.prec == P_BF16X2) {
        const uint32_t l = f2bf(f - bf2f(h));
        ((uint16_t*)a.xl)[o] = (uint16_t)l;
        st += (double)bf2f(l);
      }
      sq += st * st;
    }
  }
  sq = wave_sum(sq);
  if (lane == 0) {
    a.mu[r] = mu;
    a.isd[r] = inv;
    a.rowc[r] = sq;
  }
  if (bad) a.sc->nonfinite = 1;
}

// ---------------------------------------------------------------------------
// Random orthonormal start drawn by the library (Algorithm 1 initialisation
// when the caller passes no W0): the A records of subject i receive a v_i x k
// Gaussian G, and the first E-step takes P_i = (G^T G)^-1/2, so that the
// deferred map W_i = G P_i is the polar factor of G (Haar distributed).
// Element e = r k + b of G is normal number e % 4 of the Philox4x64-10 block
// with counter (e / 4, i, 0, 0) and key (seed, 0) (Salmon et al., SC 2011),
// by the Box-Muller transform of the block's words taken as uniforms
// u = (x / 2^11 + 1/2) 2^-53:
//   (x0, x1) -> sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1),
//   (x2, x3) -> sqrt(-2 ln u2) (cos 2 pi u3, sin 2 pi u3).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
    const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

__device__ __forceinline__ double seeded_normal(uint64_t seed, int subj, uint64_t e) {
  uint64_t c[4] = {e >> 2, (uint64_t)subj, 0, 0};
  philox4x64_10(c, seed, 0);
  const int j = (int)(e & 3);
  const uint64_t xr = (j < 2) ? c[0] : c[2];
  const uint64_t xa = (j < 2) ? c[1] : c[3];
  const double ur = ((double)(xr >> 11) + 0.5) * 0x1p-53;
  const double ua = ((double)(xa >> 11) + 0.5) * 0x1p-53;
  double sn, cs;
  sincospi(2.0 * ua, &sn, &cs);
  return sqrt(-2.0 * log(ur)) * ((j & 1) ? sn : cs);
}

template <int KP>
__global__ __launch_bounds__(256) void k_seed_a(SeedArgs a) {
  constexpr int NB = KP / 16;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)a.vp * KP) return;
  const int64_t r = idx / KP;
  const int b = (int)(idx % KP);
  float f = 0.f;
  if (r < a.v && b < a.k) f = (float)seeded_normal(a.seed, a.subj, (uint64_t)r * a.k + b);
  // A-record position of (global row R, feature b)
  const int64_t R = a.row0 + r;
  const int64_t rb = R >> 5;
  const int rr = (int)(R & 31);
  const int g = (rr & 15) >> 2, e = ((rr >> 4) << 2) + (rr & 3);
  const int lane = (b & 15) + 16 * g;
  const int64_t o = ((rb * NB + (b >> 4)) * 64 + lane) * 8 + e;
  if (a.prec == P_FP32) {
    ((float*)a.ah)[o] = f;
  } else {
    const uint32_t h = f2bf(f);
    ((uint16_t*)a.ah)[o] = (uint16_t)h;
    ((uint16_t*)a.al)[o] = (uint16_t)f2bf(f - bf2f(h));
  }
}

// c_i = ||Xhat_i||_F^2 from the per-row sums (fixed order).
__global__ __launch_bounds__(256) void k_rowsum(const double* rowc,
                                                const Subject* subj,
                                                double* c) {
  __shared__ double red[4];
  const Subject s = subj[blockIdx.x];
  double acc = 0.0;
  for (int r = threadIdx.x; r < s.vp; r += 256) acc += rowc[s.row0 + r];
  acc = block_sum256(acc, red);
  if (threadIdx.x == 0) c[blockIdx.x] = acc;
}

// ---------------------------------------------------------------------------
// M-phase, FP32 storage: A = Xhat S^T over all subjects' rows (one grouped
// launch).  Workgroup = 4 waves; each wave owns 64-row tiles (4 MFMA row
// blocks) and the full K (= features, padded) width; TRs are the contraction.
// ---------------------------------------------------------------------------

template <int KP, int PREC>
__global__ __launch_bounds__(256) void k_mphase(MArgs a) {
  if (a.sc->status) return;  // an earlier step of this iteration failed
  static_assert(PREC == P_FP32, "the BF16 forms run k_mphase_s");
  constexpr int NB = KP / 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const int64_t tb0 = (int64_t)blockIdx.x * a.tiles_per_wg;
  int64_t te = tb0 + a.tiles_per_wg;
  if (te > a.ntiles) te = a.ntiles;
  for (int64_t tile = tb0 + wave; tile < te; tile += 4) {
    const int64_t rowt = a.row_begin + tile * 64;
    const bool h1 = rowt + 32 < a.row_end;  // second 32-row half valid
    f32x4 acc[4][NB];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) acc[mb][jb] = f32x4{0.f, 0.f, 0.f, 0.f};

    // Operands of step tb + 1 are loaded while step tb's products run
    // (double buffer).
    {
      const float* X = (const float*)a.xh + rowt * a.ldt;  // uniform
      const int ld = (int)a.ldt;
      const int nstep = ld / 16;
      float4 x4[2][4], s4[2][NB];
      auto load = [&](int tb, int b) __attribute__((always_inline)) {
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          if (mb < 2 || h1)
            x4[b][mb] = *(const float4*)(X + (16 * mb + n) * ld + 16 * tb + 4 * g);
          else
            x4[b][mb] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        const float4* SR = (const float4*)a.sh + tb * NB * 64;
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) s4[b][jb] = SR[jb * 64 + lane];
      };
      auto comp = [&](int b) __attribute__((always_inline)) {
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
          if (mb >= 2 && !h1) continue;
#pragma unroll
          for (int jb = 0; jb < NB; ++jb) {
            acc[mb][jb] = mfma_f32(x4[b][mb].x, s4[b][jb].x, acc[mb][jb]);
            acc[mb][jb] = mfma_f32(x4[b][mb].y, s4[b][jb].y, acc[mb][jb]);
            acc[mb][jb] = mfma_f32(x4[b][mb].z, s4[b][jb].z, acc[mb][jb]);
            acc[mb][jb] = mfma_f32(x4[b][mb].w, s4[b][jb].w, acc[mb][jb]);
          }
        }
      };
      load(0, 0);
      for (int tb = 0; tb < nstep; tb += 2) {
        if (tb + 1 < nstep) load(tb + 1, 1);
        comp(0);
        if (tb + 1 >= nstep) break;
        if (tb + 2 < nstep) load(tb + 2, 0);
        comp(1);
      }
    }
    // Accumulator lane l holds A[rowt + 16 mb + 4 g + i][16 jb + n]; two
    // stacked row blocks are exactly one A record.
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && !h1) break;
      const int64_t rb = rowt / 32 + h;
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = acc[2 * h + (e >> 2)][jb][e & 3];
        const int64_t rec = (rb * NB + jb) * 64 + lane;
        float4* AR = (float4*)a.ah;
        AR[rec * 2] = make_float4(v[0], v[1], v[2], v[3]);
        AR[rec * 2 + 1] = make_float4(v[4], v[5], v[6], v[7]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// M-phase, BF16 forms: A = Xhat S^T as k_mphase (a wave's tile is 64 rows,
// a step 32 TRs), with the S operands of each step shared by the
// workgroup's four waves through LDS (two slots, one barrier per step)
// instead of each wave reading them from L2.  That quarters the S loads per
// Xhat byte, which compete with the Xhat loads for the CU's memory pipeline,
// and leaves a wave few enough registers (accumulators, double-buffered Xhat
// operands, the S staging) for two workgroups to share a CU.  Every wave of
// a workgroup runs the same rounds of tiles and steps (a wave without a tile
// in the last round only helps stage S), so the barriers match.
// ---------------------------------------------------------------------------

template <int KP, int PREC>
__global__ __launch_bounds__(256, 2) void k_mphase_s(MArgs a) {
  if (a.sc->status) return;  // an earlier step of this iteration failed
  static_assert(PREC != P_FP32, "BF16 forms only");
  constexpr bool X2 = PREC == P_BF16X2;
  constexpr int NB = KP / 16;
  constexpr int NS = 2 * NB * 64;            // S records of one step (uint4)
  constexpr int NSU = (NS + 255) / 256;      // staged per thread
  __shared__ uint4 Ss[2][NS];                // [slot][plane][block][lane]
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int n = lane & 15, g = lane >> 4;
  const int64_t tb0 = (int64_t)blockIdx.x * a.tiles_per_wg;
  int64_t te = tb0 + a.tiles_per_wg;
  if (te > a.ntiles) te = a.ntiles;
  if (te <= tb0) return;  // whole workgroup
  const int nround = (int)((te - tb0 + 3) / 4);
  const int ld = (int)a.ldt;
  const int nstep = ld / 32;
  const uint4* SH = (const uint4*)a.sh;
  const uint4* SL = (const uint4*)a.sl;

  // S of step tb: records [tb][block][lane] of each plane, staged through
  // registers (thread tid carries entries tid + 256 u) into a slot.
  uint4 st[NSU];
  auto s_load = [&](int tb) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < NSU; ++u) {
      const int idx = tid + 256 * u;
      st[u] = make_uint4(0, 0, 0, 0);
      if (NS % 256 == 0 || idx < NS) {
        const int pl = idx / (NB * 64), e = idx % (NB * 64);
        st[u] = (pl ? SL : SH)[(int64_t)tb * NB * 64 + e];
      }
    }
  };
  auto s_store = [&](int b) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < NSU; ++u) {
      const int idx = tid + 256 * u;
      if (NS % 256 == 0 || idx < NS) Ss[b][idx] = st[u];
    }
  };
  s_load(0);
  s_store(0);
  __syncthreads();
  int slot = 0;

  for (int rd = 0; rd < nround; ++rd) {
    const int64_t tile = tb0 + 4 * rd + wave;
    const bool valid = tile < te;
    const int64_t rowt = a.row_begin + (valid ? tile : tb0) * 64;
    const bool h1 = valid && rowt + 32 < a.row_end;  // second 32-row half valid
    f32x4 acc[4][NB];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) acc[mb][jb] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t* XH = (const uint16_t*)a.xh + rowt * a.ldt;  // uniform
    const uint16_t* XL = (const uint16_t*)a.xl + rowt * a.ldt;
    uint4 xh4[2][4], xl4[2][4];
    auto load_x = [&](int tb, int b) __attribute__((always_inline)) {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        const int o = (16 * mb + n) * ld + 32 * tb + 8 * g;
        if (valid && (mb < 2 || h1)) {
          xh4[b][mb] = *(const uint4*)(XH + o);
          if constexpr (X2) xl4[b][mb] = *(const uint4*)(XL + o);
        } else {
          xh4[b][mb] = make_uint4(0, 0, 0, 0);
          if constexpr (X2) xl4[b][mb] = make_uint4(0, 0, 0, 0);
        }
      }
    };
    // One step: stage the next step's S (after a round's last step, step 0
    // again for the next round), load the next Xhat operands, the products
    // of step tb with S from slot `slot`, then hand the next slot over at
    // the barrier.
    auto step = [&](int tb, int b) __attribute__((always_inline)) {
      s_load(tb + 1 < nstep ? tb + 1 : 0);
      if (tb + 1 < nstep) load_x(tb + 1, b ^ 1);
      if (valid) {
        const uint4* S0 = &Ss[slot][0];
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
          const uint4 sh = S0[jb * 64 + lane], sl = S0[(NB + jb) * 64 + lane];
#pragma unroll
          for (int mb = 0; mb < 4; ++mb) {
            if (mb >= 2 && !h1) continue;
            acc[mb][jb] = mfma_bf16(xh4[b][mb], sh, acc[mb][jb]);
            acc[mb][jb] = mfma_bf16(xh4[b][mb], sl, acc[mb][jb]);
            if constexpr (X2) acc[mb][jb] = mfma_bf16(xl4[b][mb], sh, acc[mb][jb]);
          }
        }
      }
      s_store(slot ^ 1);
      __syncthreads();
      slot ^= 1;
    };
    load_x(0, 0);
    for (int tb = 0; tb < nstep; tb += 2) {
      step(tb, 0);
      if (tb + 1 >= nstep) break;
      step(tb + 1, 1);
    }
    if (!valid) continue;
    // Accumulator lane l holds A[rowt + 16 mb + 4 g + i][16 jb + n]; two
    // stacked row blocks are exactly one A record.
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 1 && !h1) break;
      const int64_t rb = rowt / 32 + h;
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = acc[2 * h + (e >> 2)][jb][e & 3];
        const int64_t rec = (rb * NB + jb) * 64 + lane;
        uint4 hi, lo;
        split8(v, hi, lo);
        ((uint4*)a.ah)[rec] = hi;
        ((uint4*)a.al)[rec] = lo;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// E-phase, FP32 storage: per slice s (rows of one subject),
// Z_s = A_s^T Xhat_s (KP x ldt) and, for the M-step, G_s = A_s^T A_s (upper
// 16x16 tiles).  Workgroup = 4 waves, each wave a 64-TR column panel; rows
// are the contraction.
// Workgroup w owns an equal share of all rows (split at subject boundaries
// into slices); the npanel column panels of a row range sit on one XCD.
// ---------------------------------------------------------------------------

template <int KP, int PREC>
__global__ __launch_bounds__(256) void k_ephase(EArgs a) {
  if (a.sc->status) return;
  static_assert(PREC == P_FP32, "the BF16 forms run k_ephase_s");
  constexpr int NB = KP / 16;
  constexpr int NPAIR = NB * (NB + 1) / 2;
  constexpr int NG = (NPAIR + 3) / 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  const int range = w / a.npanel, panel = w % a.npanel;
  const int64_t cbase = (int64_t)panel * 256 + wave * 64;
  const bool do_z = cbase < a.ldt;
  const bool do_g = a.want_gram && panel == 0;
  if (!do_z && !do_g) return;
  const int sb = a.range_slice[range], se = a.range_slice[range + 1];

  for (int s = sb; s < se; ++s) {
    const Slice sl = a.slices[s];
    f32x4 acc[NB][4];
    f32x4 gacc[NG];
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[jb][q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < NG; ++p) gacc[p] = f32x4{0.f, 0.f, 0.f, 0.f};

    // Operands of the next step are loaded while the current step's
    // products run (double buffer).  Steps are 16-row halves of the 32-row
    // A records.
    const int ld = (int)a.ldt;
    {
      const int nstep = sl.nrows / 16;
      float4 av[2][NB], xv[2][4];
      auto load = [&](int hs, int b) __attribute__((always_inline)) {
        const int64_t row0 = sl.row0 + 32 * (hs >> 1);
        const int h = hs & 1;
        const float4* AR = (const float4*)a.ah + (row0 / 32) * NB * 128;  // uniform
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) av[b][jb] = AR[(jb * 64 + lane) * 2 + h];
        if (do_z) {
          const float* X = (const float*)a.xh + row0 * a.ldt + cbase;
#pragma unroll
          for (int i = 0; i < 4; ++i)
            xv[b][i] = *(const float4*)(X + (16 * h + 4 * g + i) * ld + 4 * n);
        }
      };
      auto comp = [&](int b) __attribute__((always_inline)) {
        if (do_z) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
              const float ae = ((const float*)&av[b][jb])[i];
              acc[jb][0] = mfma_f32(ae, xv[b][i].x, acc[jb][0]);
              acc[jb][1] = mfma_f32(ae, xv[b][i].y, acc[jb][1]);
              acc[jb][2] = mfma_f32(ae, xv[b][i].z, acc[jb][2]);
              acc[jb][3] = mfma_f32(ae, xv[b][i].w, acc[jb][3]);
            }
        }
        if (do_g) {
          int p = 0;
#pragma unroll
          for (int j1 = 0; j1 < NB; ++j1)
#pragma unroll
            for (int j2 = j1; j2 < NB; ++j2, ++p)
              if ((p & 3) == wave)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  gacc[p >> 2] = mfma_f32(((const float*)&av[b][j1])[i],
                                          ((const float*)&av[b][j2])[i], gacc[p >> 2]);
        }
      };
      if (nstep > 0) load(0, 0);
      for (int hs = 0; hs < nstep; hs += 2) {
        if (hs + 1 < nstep) load(hs + 1, 1);
        comp(0);
        if (hs + 1 >= nstep) break;
        if (hs + 2 < nstep) load(hs + 2, 0);
        comp(1);
      }
    }
    // Z tile: lane holds Z[16 jb + 4 g + i][cbase + 4 n + q].
    if (do_z) {
      float* zp = a.zpart + (int64_t)s * KP * a.ldt + cbase;  // uniform
#pragma unroll
      for (int jb = 0; jb < NB; ++jb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = 16 * jb + 4 * g + i;
          *(float4*)(zp + j * ld + 4 * n) =
              make_float4(acc[jb][0][i], acc[jb][1][i], acc[jb][2][i],
                          acc[jb][3][i]);
        }
    }
    if (do_g) {
      float* gp = a.gpart + (int64_t)s * KP * KP;
      int p = 0;
#pragma unroll
      for (int j1 = 0; j1 < NB; ++j1)
#pragma unroll
        for (int j2 = j1; j2 < NB; ++j2, ++p)
          if ((p & 3) == wave)
#pragma unroll
            for (int i = 0; i < 4; ++i)
              gp[(16 * j1 + 4 * g + i) * KP + 16 * j2 + n] = gacc[p >> 2][i];
    }
  }
}


// ---------------------------------------------------------------------------
// E-phase, BF16 forms: Z_s = A_s^T Xhat_s and G_s = A_s^T A_s as k_ephase,
// with both operands staged in LDS by direct loads one 32-row block ahead
// (double buffer): the block of Xhat (32 rows x the workgroup's 512-TR
// panel, records as in k_staged) and the block's A records, which the eight
// waves share instead of each reading them from L2.  The rows-as-K operand
// of Xhat comes from transposing LDS reads, so a wave holds no Xhat in
// registers and two waves fit a SIMD.  Wave w adds TRs 64 w .. 64 w + 63 of
// the panel and its share of the Gram tiles (panel 0).  One barrier per
// block: after it the block's loads have landed for every wave, and every
// wave is done with the buffer the next loads refill.
// ---------------------------------------------------------------------------

constexpr int kEphasePanel = 512;  // TRs per k_ephase_s workgroup

template <int KP, int PREC>
__global__ __launch_bounds__(512) void k_ephase_s(EArgs a) {
  if (a.sc->status) return;  // an earlier step of this iteration failed
  static_assert(PREC != P_FP32, "BF16 forms only");
  constexpr bool X2 = PREC == P_BF16X2;
  constexpr int PL = X2 ? 2 : 1;
  constexpr int NW = 8;
  constexpr int NB = KP / 16;
  constexpr int NSTEP = kEphasePanel / 32;   // 32-TR steps of a panel
  constexpr int NREC = PL * 2 * NSTEP;       // Xhat records per block
  constexpr int LPW = NREC / NW;             // Xhat loads per wave per block
  constexpr int NGRP = 4, LPG = LPW / NGRP;
  static_assert(LPW % NGRP == 0, "");
  constexpr int NAR = 2 * NB;                // A records per block (hi, lo)
  constexpr int NPAIR = NB * (NB + 1) / 2;
  constexpr int NG = (NPAIR + NW - 1) / NW;
  __shared__ uint4 Xs[2][NREC][64];
  __shared__ uint4 As[2][NAR][64];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  const int range = w / a.npanel, panel = w % a.npanel;
  const int64_t ldt = a.ldt;
  const int64_t c0 = (int64_t)panel * kEphasePanel;   // first TR of the panel
  const int64_t nin = (ldt - c0) / 32;
  const int nst = nin < NSTEP ? (int)nin : NSTEP;  // steps inside ldt
  const bool do_z = 64 * wave < 32 * nst;
  const bool do_g = a.want_gram && panel == 0;
  const int sb = a.range_slice[range], se = a.range_slice[range + 1];
  if (sb >= se) return;  // whole workgroup
  const uint16_t* XH = (const uint16_t*)a.xh;
  const uint16_t* XL = (const uint16_t*)a.xl;
  const uint4* AH = (const uint4*)a.ah;
  const uint4* AL = (const uint4*)a.al;

  // Loads of the block at global row r0 into buffer b: Xhat records r =
  // w LPW .. w LPW + LPW - 1 in NGRP groups (records of steps beyond ldt are
  // not loaded; only waves without TRs there would read them), A records
  // w, w + NW, ... with group 0.
  const int voff_lane = (int)((n * ldt + 8 * g) * 2);
  auto issue = [&](int64_t r0, int b, int grp) __attribute__((always_inline)) {
    const uint32_t xbytes = (uint32_t)((32 * ldt - c0) * 2);
    const v4i_rsrc RH = make_rsrc_v4(XH + r0 * ldt + c0, xbytes);
    const v4i_rsrc RL = make_rsrc_v4(XL + r0 * ldt + c0, xbytes);
#pragma unroll
    for (int jj = 0; jj < LPG; ++jj) {
      const int r = wave * LPW + grp * LPG + jj;
      const int pl = r / (2 * NSTEP), rb = (r / NSTEP) & 1, st = r % NSTEP;
      if (st < nst)
        load_lds16(pl ? RL : RH, &Xs[b][r][0], voff_lane, (int)((16 * rb * ldt + 32 * st) * 2));
    }
    if (grp == 0) {
      const int64_t rb = r0 / 32;
      const v4i_rsrc QH = make_rsrc_v4(AH + rb * NB * 64, NB * 1024);
      const v4i_rsrc QL = make_rsrc_v4(AL + rb * NB * 64, NB * 1024);
#pragma unroll
      for (int r = wave; r < NAR; r += NW)
        load_lds16(r < NB ? QH : QL, &As[b][r][0], lane * 16, (r % NB) * 1024);
    }
  };
  auto rec = [](int pl, int rb, int st) { return (pl * 2 + rb) * NSTEP + st; };

  f32x4 zacc[NB][4];
  f32x4 gacc[NG];
#pragma unroll
  for (int jb = 0; jb < NB; ++jb)
#pragma unroll
    for (int q = 0; q < 4; ++q) zacc[jb][q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int p = 0; p < NG; ++p) gacc[p] = f32x4{0.f, 0.f, 0.f, 0.f};

  int s = sb, cr = 0, buf = 0;
  int64_t row0;
  int32_t nrows;
  slice_s(a.slices + s, row0, nrows);
#pragma unroll
  for (int grp = 0; grp < NGRP; ++grp) issue(row0, 0, grp);
  // Transposing reads: lane 4r + q of group g reads TRs 4q..4q+3 of rows
  // 4g + r (first read) and 16 + 4g + r (second read) of a 16-TR tile.
  const int tr_r = (lane & 15) >> 2, tr_q = lane & 3;
  for (;;) {
    int ns = s, ncr = cr + 32;
    if (ncr >= nrows) { ns = s + 1; ncr = 0; }
    const bool has_next = ns < se;
    int64_t nrow0 = row0;
    int32_t nnrows = nrows;
    if (has_next && ns != s) slice_s(a.slices + ns, nrow0, nnrows);
    const int64_t nr0 = nrow0 + ncr;  // the next block's first row
    __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8));  // vmcnt(0)
    __syncthreads();
    if (has_next) issue(nr0, buf ^ 1, 0);
    if (do_z) {
      // Xhat operands of the wave's four 16-TR tiles, then the products
      // block by block of features (A operands: record jb (hi) and NB + jb
      // (lo), in lane order)
      const char* xb0 = (const char*)&Xs[buf][0][0];
      uint4 bh[4], bl[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int t = 64 * wave + 16 * q + 4 * tr_q;  // first of this lane's 4 TRs
        const int st = t >> 5, gq = (t & 31) >> 3, half = (t & 7) >> 2;
        const int in_rec = ((4 * g + tr_r) + 16 * gq) * 16 + 8 * half;
        bh[q] = pack_tr(ds_tr16(xb0 + rec(0, 0, st) * 1024 + in_rec),
                        ds_tr16(xb0 + rec(0, 1, st) * 1024 + in_rec));
        if constexpr (X2)
          bl[q] = pack_tr(ds_tr16(xb0 + rec(1, 0, st) * 1024 + in_rec),
                          ds_tr16(xb0 + rec(1, 1, st) * 1024 + in_rec));
      }
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
        const uint4 ah = As[buf][jb][lane], al = As[buf][NB + jb][lane];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          zacc[jb][q] = mfma_bf16(ah, bh[q], zacc[jb][q]);
          zacc[jb][q] = mfma_bf16(al, bh[q], zacc[jb][q]);
          if constexpr (X2) zacc[jb][q] = mfma_bf16(ah, bl[q], zacc[jb][q]);
        }
#pragma unroll
        for (int grp = 1; grp < NGRP; ++grp)
          if (jb == (grp * NB) / NGRP && has_next) issue(nr0, buf ^ 1, grp);
        // keeps the scheduler from reading every block's A ahead (registers)
        __builtin_amdgcn_sched_barrier(0);
      }
    } else if (has_next) {
#pragma unroll
      for (int grp = 1; grp < NGRP; ++grp) issue(nr0, buf ^ 1, grp);
    }
    if (do_g) {
      int p = 0;
#pragma unroll
      for (int j1 = 0; j1 < NB; ++j1)
#pragma unroll
        for (int j2 = j1; j2 < NB; ++j2, ++p)
          if ((p % NW) == wave) {
            const uint4 h1 = As[buf][j1][lane], l1 = As[buf][NB + j1][lane];
            const uint4 h2 = As[buf][j2][lane], l2 = As[buf][NB + j2][lane];
            gacc[p / NW] = mfma_bf16(h1, h2, gacc[p / NW]);
            gacc[p / NW] = mfma_bf16(h1, l2, gacc[p / NW]);
            gacc[p / NW] = mfma_bf16(l1, h2, gacc[p / NW]);
            // lo*lo too: its error would scale with cond(A^T A) in W^T W.
            gacc[p / NW] = mfma_bf16(l1, l2, gacc[p / NW]);
          }
    }
    if (ns != s || !has_next) {
      // the slice is complete: lane holds Z[16 jb + 4 g + i][c0 + 64 w + 16 q + n]
      if (do_z) {
        // one feature row at a time (its offset is wave-uniform), so that
        // the compiler does not keep every element's address live in the loop
        float* zp = a.zpart + (int64_t)s * KP * ldt + c0 + 64 * wave + n + 4 * g * ldt;
#pragma unroll
        for (int jb = 0; jb < NB; ++jb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float* zr = zp + (int64_t)__builtin_amdgcn_readfirstlane((16 * jb + i) * (int)ldt);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              zr[16 * q] = zacc[jb][q][i];
              zacc[jb][q][i] = 0.f;
            }
          }
      }
      if (do_g) {
        float* gp = a.gpart + (int64_t)s * KP * KP;
        int p = 0;
#pragma unroll
        for (int j1 = 0; j1 < NB; ++j1)
#pragma unroll
          for (int j2 = j1; j2 < NB; ++j2, ++p)
            if ((p % NW) == wave)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                gp[(16 * j1 + 4 * g + i) * KP + 16 * j2 + n] = gacc[p / NW][i];
                gacc[p / NW][i] = 0.f;
              }
      }
    }
    if (!has_next) break;
    s = ns;
    cr = ncr;
    row0 = nrow0;
    nrows = nnrows;
    buf ^= 1;
  }
}

// ---------------------------------------------------------------------------
// One-pass sweep (BF16 forms, K padding <= 64, ldt in {128, 256, 384, 512}):
// A = Xhat S^T never goes to HBM.  Workgroup = NW = ldt / 64 waves with all
// of S (bf16 hi+lo records) resident in LDS for the whole launch.  Each
// slice is walked in chunks of CH rows (16 NW; 64 with eight waves):
//   part 1: wave w < CH / 16 forms the 16-row block w of A over all TRs,
//           all features; its Xhat rows stream from HBM through a 4-deep
//           register ring, S operands come from LDS one step ahead; the
//           bf16 hi+lo result is written into the chunk's A records in LDS;
//   part 2: after one barrier, wave w adds A^T Xhat[:, 64 w .. 64 w + 63]
//           over the chunk into its Z columns (reading the chunk's Xhat a
//           second time, from the caches where it is still resident) and
//           its share of the Gram tiles A^T A.
// Z_s and G_s per slice equal what the two-pass E-phase forms from
// A = Xhat S^T; A itself never goes to HBM.
// ---------------------------------------------------------------------------
template <int KP, int PREC, int NW, int CH>
__global__ __launch_bounds__(NW * 64) void k_fused(FusedArgs a) {
  if (a.sc->status) return;
  static_assert(PREC != P_FP32, "one-pass sweep is for the BF16 forms");
  static_assert(NW % 2 == 0, "chunks are whole 32-row A records");
  constexpr bool X2 = PREC == P_BF16X2;
  constexpr int NB = KP / 16;
  constexpr int NPAIR = NB * (NB + 1) / 2;
  constexpr int NG = (NPAIR + NW - 1) / NW;
  constexpr int LDT = 64 * NW;
  constexpr int NSTEP = LDT / 32;  // 32-TR MFMA steps
  // Chunk rows CH: one 16-row block per wave (CH = 16 NW), or with eight
  // waves also 64-row chunks, in which half of them form A: the smaller
  // chunk keeps the lines that part 2 reads again within reach of the L2.
  static_assert(CH % 32 == 0 && CH <= 16 * NW, "chunks are whole A records");
  constexpr int NPW = CH / 16;     // waves with part-1 work
  constexpr int NRB = CH / 32;     // A records (32-row blocks) per chunk
  constexpr int D = 4;             // Xhat prefetch depth in part 1
  __shared__ uint4 SHs[NSTEP][NB][64];
  __shared__ uint4 SLs[NSTEP][NB][64];
  __shared__ uint2 ARH[NRB][NB][64][2];  // [.][.][lane][row half]
  __shared__ uint2 ARL[NRB][NB][64][2];
  // readfirstlane: the wave index (and every buffer descriptor built from it)
  // is wave-uniform, so descriptors live in scalar registers.
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const uint16_t* XH = (const uint16_t*)a.xh;
  const uint16_t* XL = (const uint16_t*)a.xl;
  const int c0 = 64 * wave;

  // S records (current posterior mean) -> LDS, once.
  for (int r = threadIdx.x; r < NSTEP * NB * 64; r += NW * 64) {
    (&SHs[0][0][0])[r] = ((const uint4*)a.sh)[r];
    (&SLs[0][0][0])[r] = ((const uint4*)a.sl)[r];
  }
  __syncthreads();

  const int sb = a.range_slice[blockIdx.x], se = a.range_slice[blockIdx.x + 1];
  for (int s = sb; s < se; ++s) {
    const Slice sc = a.slices[s];
    f32x4 zacc[NB][4];
    f32x4 gacc[NG];
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int q = 0; q < 4; ++q) zacc[jb][q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int p = 0; p < NG; ++p) gacc[p] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int cr = 0; cr < sc.nrows; cr += CH) {
      const int nrow = min(CH, sc.nrows - cr);  // multiple of 32
      const int64_t rc = sc.row0 + cr;
      // ---- part 1: rows [16 rw, 16 rw + 16), all feature blocks
      const int rw = wave;
      if (wave < NPW && 16 * rw < nrow) {
        const uint32_t wbytes = 16u * LDT * 2u;
        const auto RH = make_rsrc(XH + (rc + 16 * rw) * LDT, wbytes);
        const auto RL = make_rsrc(XL + (rc + 16 * rw) * LDT, wbytes);
        const int vx = (n * LDT + 8 * g) * 2;
        f32x4 acc[NB];
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) acc[jb] = f32x4{0.f, 0.f, 0.f, 0.f};
        uint4 xh[D], xl[D];
#pragma unroll
        for (int st = 0; st < D && st < NSTEP; ++st) {
          xh[st] = bload16(RH, vx, st * 64);
          if constexpr (X2) xl[st] = bload16(RL, vx, st * 64);
        }
        // S operands are read from LDS one step ahead (double buffer) so
        // their latency hides behind the previous step's products.
        uint4 th[2][NB], tl[2][NB];
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) {
          th[0][jj] = SHs[0][jj][lane];
          tl[0][jj] = SLs[0][jj][lane];
        }
#pragma unroll
        for (int tb = 0; tb < NSTEP; ++tb) {
          const int st = tb % D, sb2 = tb & 1;
          if (tb + 1 < NSTEP) {
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) {
              th[sb2 ^ 1][jj] = SHs[tb + 1][jj][lane];
              tl[sb2 ^ 1][jj] = SLs[tb + 1][jj][lane];
            }
          }
          const uint4 xa = xh[st];
          uint4 xb;
          if constexpr (X2) xb = xl[st];
          if (tb + D < NSTEP) {  // refill this ring slot
            xh[st] = bload16(RH, vx, (tb + D) * 64);
            if constexpr (X2) xl[st] = bload16(RL, vx, (tb + D) * 64);
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int jj = 0; jj < NB; ++jj) {
            acc[jj] = mfma_bf16(xa, th[sb2][jj], acc[jj]);
            acc[jj] = mfma_bf16(xa, tl[sb2][jj], acc[jj]);
            if constexpr (X2) acc[jj] = mfma_bf16(xb, th[sb2][jj], acc[jj]);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        // lane holds A[16 rw + 4 g + i][16 jb + n]: half of an A record
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
          uint32_t h01, l01, h23, l23;
          split2(acc[jb][0], acc[jb][1], h01, l01);
          split2(acc[jb][2], acc[jb][3], h23, l23);
          ARH[rw >> 1][jb][lane][rw & 1] = make_uint2(h01, h23);
          ARL[rw >> 1][jb][lane][rw & 1] = make_uint2(l01, l23);
        }
      }
      __syncthreads();
      // ---- part 2: Z[:, 64 w ..] += A^T Xhat, Gram tiles
      {
        const int nblk = nrow / 32;
        const uint32_t cbytes = (uint32_t)nrow * LDT * 2u;
        const auto RH = make_rsrc(XH + rc * LDT + c0, cbytes);
        const auto RL = make_rsrc(XL + rc * LDT + c0, cbytes);
        const int vx = (4 * g * LDT + 4 * n) * 2;
        uint2 xv[2][8], xw[2][8];
        auto load = [&](int b, int buf) {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int so = (32 * b + (e & 3) + 16 * (e >> 2)) * LDT * 2;
            xv[buf][e] = bload8(RH, vx, so);
            if constexpr (X2) xw[buf][e] = bload8(RL, vx, so);
          }
        };
        auto block = [&](int b, int buf) {
          uint4 ah[NB], al[NB];
#pragma unroll
          for (int jb = 0; jb < NB; ++jb) {
            const uint2 h0 = ARH[b][jb][lane][0], h1 = ARH[b][jb][lane][1];
            const uint2 l0 = ARL[b][jb][lane][0], l1 = ARL[b][jb][lane][1];
            ah[jb] = make_uint4(h0.x, h0.y, h1.x, h1.y);
            al[jb] = make_uint4(l0.x, l0.y, l1.x, l1.y);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            uint4 bh, bl;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
              const uint32_t a0 = (q < 2) ? xv[buf][2 * d].x : xv[buf][2 * d].y;
              const uint32_t a1 = (q < 2) ? xv[buf][2 * d + 1].x : xv[buf][2 * d + 1].y;
              ((uint32_t*)&bh)[d] = (q & 1) ? ((a0 >> 16) | (a1 & 0xffff0000u))
                                            : ((a0 & 0xffffu) | (a1 << 16));
              if constexpr (X2) {
                const uint32_t b0 = (q < 2) ? xw[buf][2 * d].x : xw[buf][2 * d].y;
                const uint32_t b1 = (q < 2) ? xw[buf][2 * d + 1].x : xw[buf][2 * d + 1].y;
                ((uint32_t*)&bl)[d] = (q & 1) ? ((b0 >> 16) | (b1 & 0xffff0000u))
                                              : ((b0 & 0xffffu) | (b1 << 16));
              }
            }
#pragma unroll
            for (int jb = 0; jb < NB; ++jb) {
              zacc[jb][q] = mfma_bf16(ah[jb], bh, zacc[jb][q]);
              zacc[jb][q] = mfma_bf16(al[jb], bh, zacc[jb][q]);
              if constexpr (X2) zacc[jb][q] = mfma_bf16(ah[jb], bl, zacc[jb][q]);
            }
          }
          int p = 0;
#pragma unroll
          for (int j1 = 0; j1 < NB; ++j1)
#pragma unroll
            for (int j2 = j1; j2 < NB; ++j2, ++p)
              if ((p % NW) == wave) {
                gacc[p / NW] = mfma_bf16(ah[j1], ah[j2], gacc[p / NW]);
                gacc[p / NW] = mfma_bf16(ah[j1], al[j2], gacc[p / NW]);
                gacc[p / NW] = mfma_bf16(al[j1], ah[j2], gacc[p / NW]);
                gacc[p / NW] = mfma_bf16(al[j1], al[j2], gacc[p / NW]);
              }
        };
        load(0, 0);
        for (int b = 0; b < nblk; b += 2) {
          if (b + 1 < nblk) load(b + 1, 1);
          block(b, 0);
          if (b + 1 >= nblk) break;
          if (b + 2 < nblk) load(b + 2, 0);
          block(b + 1, 1);
        }
      }
      __syncthreads();
    }
    // Z tile: lane holds Z[16 jb + 4 g + i][c0 + 4 n + q].
    float* zp = a.zpart + (int64_t)s * KP * LDT + c0;  // uniform
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = 16 * jb + 4 * g + i;
        *(float4*)(zp + j * LDT + 4 * n) =
            make_float4(zacc[jb][0][i], zacc[jb][1][i], zacc[jb][2][i], zacc[jb][3][i]);
      }
    float* gp = a.gpart + (int64_t)s * KP * KP;
    int p = 0;
#pragma unroll
    for (int j1 = 0; j1 < NB; ++j1)
#pragma unroll
      for (int j2 = j1; j2 < NB; ++j2, ++p)
        if ((p % NW) == wave)
#pragma unroll
          for (int i = 0; i < 4; ++i)
            gp[(16 * j1 + 4 * g + i) * KP + 16 * j2 + n] = gacc[p / NW][i];
  }
}

// ---------------------------------------------------------------------------
// One-pass sweep with Xhat staged in LDS (BF16 forms): the same partials as
// k_fused (Z_s = A_s^T Xhat_s, G_s = A_s^T A_s per slice, A = Xhat S^T never
// stored), but every 32-row chunk of Xhat is read from HBM exactly once, by
// direct-to-LDS buffer loads issued one chunk ahead (double buffer), and both
// uses read it from LDS:
//  part 1: A[32 rows, KP] = Xhat S^T.  S lives in registers: wave w holds the
//          S operands of FPW feature blocks (group w % (NB / FPW)) for the TR
//          part w / (NB / FPW), and forms that part's partial sums for both
//          16-row tiles, reading each Xhat operand once for its FPW blocks.
//          The TR parts are added through LDS in a fixed order and rounded
//          to bf16 hi+lo A records.
//  part 2: wave w adds A^T Xhat over its 64 TRs and its share of the Gram
//          tiles.  The rows-as-K operand of Xhat comes from LDS by transposing
//          reads (ds_read_b64_tr_b16: in each 16-lane group, lane 4r + q
//          supplies TRs 4q..4q+3 of row r and every lane receives its own TR
//          of the four rows).
// LDS records: one 1 KB record per (plane, 16-row tile, 32-TR step), in the
// matrix-core operand order (lane n + 16 g holds row n, TRs 8g..8g+7), which
// is also the order a direct load deposits (lane j's 16 bytes at 16 j).
// Partial sums: one 1 KB slot per (TR part, output), an output being a
// (feature block, row tile) pair.  An output is finalised by one of the waves
// that formed a partial sum of it, which keeps that partial in registers and
// reads the other TR parts' slots; the slots so left unused hold the A
// operand records (hi and lo) of each feature block.
// ---------------------------------------------------------------------------
template <int KP, int PREC, int NW>
__global__ __launch_bounds__(NW * 64) void k_staged(FusedArgs a) {
  if (a.sc->status) return;  // no kernel of this launch raises it: uniform
  static_assert(PREC != P_FP32, "one-pass sweep is for the BF16 forms");
  constexpr bool X2 = PREC == P_BF16X2;
  constexpr int PL = X2 ? 2 : 1;
  constexpr int NB = KP / 16;
  constexpr int LDT = 64 * NW;
  constexpr int NSTEP = LDT / 32;
  constexpr int FPW = (NB % 2 == 0) ? 2 : NB;  // feature blocks per part-1 wave
  constexpr int NFG = NB / FPW;                // feature groups
  static_assert(NW % NFG == 0, "feature groups must divide the waves");
  constexpr int TP = NW / NFG;         // TR parts of part 1
  static_assert(NSTEP % TP == 0, "TR parts are whole 32-TR steps");
  constexpr int SPW = NSTEP / TP;      // part-1 steps per wave
  constexpr int NOUT = 2 * NB;         // outputs: (feature block, row tile)
  constexpr int NREC = PL * 2 * NSTEP; // records per 32-row chunk
  constexpr int LPW = NREC / NW;       // direct loads per wave per chunk
  static_assert(NREC % NW == 0 && LPW <= 15, "");
  constexpr int NPAIR = NB * (NB + 1) / 2;
  constexpr int NG = (NPAIR + NW - 1) / NW;
  __shared__ uint4 Xs[2][NREC][64];
  __shared__ uint4 Pa[TP][NOUT][64];  // [TR part][output][lane]
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const int fg = wave % NFG, tp = wave / NFG;
  const uint16_t* XH = (const uint16_t*)a.xh;
  const uint16_t* XL = (const uint16_t*)a.xl;

  const int sb = a.range_slice[blockIdx.x], se = a.range_slice[blockIdx.x + 1];
  if (sb >= se) return;

  // S operands of this wave's feature blocks and TR part (S records
  // [step][feature block][lane]).
  uint4 sh[FPW][SPW], sl[FPW][SPW];
#pragma unroll
  for (int f = 0; f < FPW; ++f)
#pragma unroll
    for (int j = 0; j < SPW; ++j) {
      const int st = tp * SPW + j, fb = fg * FPW + f;
      sh[f][j] = ((const uint4*)a.sh)[(st * NB + fb) * 64 + lane];
      sl[f][j] = ((const uint4*)a.sl)[(st * NB + fb) * 64 + lane];
    }

  // Direct loads of the chunk starting at global row r0 into buffer b:
  // wave w fetches records w LPW .. w LPW + LPW - 1, in NGRP groups issued
  // while the chunk before it is processed: after the chunk's first barrier,
  // early in part 1, at the end of part 1 and after the finalise (a wave
  // whose load cannot enter the memory pipeline stalls at the issue, so one
  // burst of all loads would hold every wave up at once; the last group
  // still lands a whole part 2 before it is needed).
  constexpr int NGRP = (LPW % 4 == 0) ? 4 : ((LPW % 2 == 0) ? 2 : 1);
  constexpr int LPG = LPW / NGRP;  // loads per group
  const int voff_lane = (n * LDT + 8 * g) * 2;
  auto issue = [&](int64_t r0, int b, int grp) {
    const uint32_t cbytes = 32u * LDT * 2u;
    const v4i_rsrc RH = make_rsrc_v4(XH + r0 * LDT, cbytes);
    const v4i_rsrc RL = make_rsrc_v4(XL + r0 * LDT, cbytes);
#pragma unroll
    for (int jj = 0; jj < LPG; ++jj) {
      const int r = wave * LPW + grp * LPG + jj;
      const int pl = r / (2 * NSTEP), rb = (r / NSTEP) & 1, st = r % NSTEP;
      const int so = (16 * rb * LDT + 32 * st) * 2;
      load_lds16(pl ? RL : RH, &Xs[b][r][0], voff_lane, so);
    }
  };
  // record index of (plane, 16-row tile, step)
  auto rec = [](int pl, int rb, int st) { return (pl * 2 + rb) * NSTEP + st; };
  // TR part whose wave finalises output o (its slot of o holds no partial)
  auto fin_part = [](int o) { return (o % (2 * FPW)) % TP; };

  f32x4 zacc[NB][4];
  f32x4 gacc[NG];
#pragma unroll
  for (int jb = 0; jb < NB; ++jb)
#pragma unroll
    for (int q = 0; q < 4; ++q) zacc[jb][q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int p = 0; p < NG; ++p) gacc[p] = f32x4{0.f, 0.f, 0.f, 0.f};

  int s = sb, cr = 0, buf = 0;
  int64_t row0;
  int32_t nrows;
  slice_s(a.slices + s, row0, nrows);
#pragma unroll
  for (int grp = 0; grp < NGRP; ++grp) issue(row0, 0, grp);
  // Part-2 transposing reads: lane 4r + q of group g reads TRs 4q..4q+3 of
  // rows 4g + r (first read) and 16 + 4g + r (second read) of a 16-TR tile.
  const int tr_r = (lane & 15) >> 2, tr_q = lane & 3;
  for (;;) {
    int ns = s, ncr = cr + 32;
    if (ncr >= nrows) { ns = s + 1; ncr = 0; }
    const bool has_next = ns < se;
    int64_t nrow0 = row0;
    int32_t nnrows = nrows;
    if (has_next && ns != s) slice_s(a.slices + ns, nrow0, nnrows);
    const int64_t nr0 = nrow0 + ncr;  // the next chunk's first row
    // This chunk's loads (issued during the previous one) have landed, for
    // every wave after the barrier; it also marks every wave done with the
    // previous chunk, whose buffer the next chunk's loads then refill.
    __builtin_amdgcn_s_waitcnt(0 | (7 << 4) | (15 << 8));
    __syncthreads();
    if (has_next) issue(nr0, buf ^ 1, 0);
    // ---- part 1: partial A over this wave's TR part, its feature blocks
    {
      f32x4 acc[FPW][2];
#pragma unroll
      for (int f = 0; f < FPW; ++f)
#pragma unroll
        for (int m = 0; m < 2; ++m) acc[f][m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < SPW; ++j) {
        const int st = tp * SPW + j;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          const uint4 xa = Xs[buf][rec(0, m, st)][lane];
          uint4 xb;
          if constexpr (X2) xb = Xs[buf][rec(1, m, st)][lane];
#pragma unroll
          for (int f = 0; f < FPW; ++f) {
            acc[f][m] = mfma_bf16(xa, sh[f][j], acc[f][m]);
            acc[f][m] = mfma_bf16(xa, sl[f][j], acc[f][m]);
            if constexpr (X2) acc[f][m] = mfma_bf16(xb, sh[f][j], acc[f][m]);
          }
        }
        if (NGRP > 1 && has_next && j == SPW / 4) issue(nr0, buf ^ 1, 1);
        if (NGRP > 2 && has_next && j == SPW - 1) issue(nr0, buf ^ 1, 2);
      }
      // Output o = 2 FPW fg + r (r = 2 f + m: feature block FPW fg + f, row
      // tile m) is finalised by the wave of TR part r % TP in feature group
      // fg, which keeps its own partial sum in registers; the other TR parts
      // pass theirs through their slots.
#pragma unroll
      for (int f = 0; f < FPW; ++f)
#pragma unroll
        for (int m = 0; m < 2; ++m)
          if ((2 * f + m) % TP != tp)
            Pa[tp][2 * (fg * FPW + f) + m][lane] =
                make_uint4(__float_as_uint(acc[f][m][0]), __float_as_uint(acc[f][m][1]),
                           __float_as_uint(acc[f][m][2]), __float_as_uint(acc[f][m][3]));
      __syncthreads();
      // The finaliser adds the TR parts in order and rounds to hi + lo.  The A
      // operands of block fb go to the two slots that hold no partial sum,
      // those of outputs 2 fb (hi) and 2 fb + 1 (lo), as whole operand
      // records: lane l's 16 bytes are its pair of row tile 0, then of row
      // tile 1, so output 2 fb + m writes bytes 8 m .. 8 m + 7 of each lane.
#pragma unroll
      for (int f = 0; f < FPW; ++f)
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          if ((2 * f + m) % TP != tp) continue;
          const int fb = fg * FPW + f, o = 2 * fb + m;
          uint4 u[TP];  // the other TR parts' slots, read before any is used
#pragma unroll
          for (int p = 0; p < TP; ++p)
            if (p != tp) u[p] = Pa[p][o][lane];
          float v[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int p = 0; p < TP; ++p) {
            if (p == tp) {
#pragma unroll
              for (int i = 0; i < 4; ++i) v[i] += acc[f][m][i];
            } else {
              v[0] += __uint_as_float(u[p].x);
              v[1] += __uint_as_float(u[p].y);
              v[2] += __uint_as_float(u[p].z);
              v[3] += __uint_as_float(u[p].w);
            }
          }
          uint32_t h01, l01, h23, l23;
          split2(v[0], v[1], h01, l01);
          split2(v[2], v[3], h23, l23);
          ((uint2*)&Pa[fin_part(2 * fb)][2 * fb][0])[2 * lane + m] = make_uint2(h01, h23);
          ((uint2*)&Pa[fin_part(2 * fb + 1)][2 * fb + 1][0])[2 * lane + m] = make_uint2(l01, l23);
        }
    }
    if (NGRP > 3 && has_next) issue(nr0, buf ^ 1, 3);
    // ---- part 2: Z[:, 64 w + 16 q + n] += A^T Xhat, Gram tiles
    {
      const char* xb0 = (const char*)&Xs[buf][0][0];
      // Xhat operands of 16-TR tile q by transposing reads
      auto load_b = [&](int q, uint4& bh, uint4& bl) {
        const int t = 64 * wave + 16 * q + 4 * tr_q;  // first of this lane's 4 TRs
        const int st = t >> 5, gq = (t & 31) >> 3, half = (t & 7) >> 2;
        const int in_rec = ((4 * g + tr_r) + 16 * gq) * 16 + 8 * half;
        {
          const v4s r1 = ds_tr16(xb0 + rec(0, 0, st) * 1024 + in_rec);
          const v4s r2 = ds_tr16(xb0 + rec(0, 1, st) * 1024 + in_rec);
          bh = pack_tr(r1, r2);
        }
        if constexpr (X2) {
          const v4s r1 = ds_tr16(xb0 + rec(1, 0, st) * 1024 + in_rec);
          const v4s r2 = ds_tr16(xb0 + rec(1, 1, st) * 1024 + in_rec);
          bl = pack_tr(r1, r2);
        }
      };
      // Tile 0's reads do not depend on the finalise, so they go out before
      // the barrier that publishes it.  LDS operations of a wave complete in
      // order: once at most those reads are outstanding, this wave's
      // finalise writes are done, which is all the barrier has to wait for.
      uint4 bh0, bl0;
      asm volatile("" ::: "memory");
      load_b(0, bh0, bl0);
      asm volatile("s_waitcnt lgkmcnt(%0)\n\ts_barrier" :: "n"(X2 ? 4 : 2) : "memory");
      // A operands of block jb: whole operand records (hi, lo)
      uint4 ah[NB], al[NB];
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
        ah[jb] = Pa[fin_part(2 * jb)][2 * jb][lane];
        al[jb] = Pa[fin_part(2 * jb + 1)][2 * jb + 1][lane];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint4 bh = bh0, bl = bl0;
        if (q > 0) load_b(q, bh, bl);
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
          zacc[jb][q] = mfma_bf16(ah[jb], bh, zacc[jb][q]);
          zacc[jb][q] = mfma_bf16(al[jb], bh, zacc[jb][q]);
          if constexpr (X2) zacc[jb][q] = mfma_bf16(ah[jb], bl, zacc[jb][q]);
        }
      }
      int p = 0;
#pragma unroll
      for (int j1 = 0; j1 < NB; ++j1)
#pragma unroll
        for (int j2 = j1; j2 < NB; ++j2, ++p)
          if ((p % NW) == wave) {
            gacc[p / NW] = mfma_bf16(ah[j1], ah[j2], gacc[p / NW]);
            gacc[p / NW] = mfma_bf16(ah[j1], al[j2], gacc[p / NW]);
            gacc[p / NW] = mfma_bf16(al[j1], ah[j2], gacc[p / NW]);
            gacc[p / NW] = mfma_bf16(al[j1], al[j2], gacc[p / NW]);
          }
    }
    if (ns != s || !has_next) {
      // the slice is complete: lane holds Z[16 jb + 4 g + i][64 w + 16 q + n]
      float* zp = a.zpart + (int64_t)s * KP * LDT + 64 * wave + n;
#pragma unroll
      for (int jb = 0; jb < NB; ++jb)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            zp[(16 * jb + 4 * g + i) * LDT + 16 * q] = zacc[jb][q][i];
            zacc[jb][q][i] = 0.f;
          }
      float* gp = a.gpart + (int64_t)s * KP * KP;
      int p = 0;
#pragma unroll
      for (int j1 = 0; j1 < NB; ++j1)
#pragma unroll
        for (int j2 = j1; j2 < NB; ++j2, ++p)
          if ((p % NW) == wave)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              gp[(16 * j1 + 4 * g + i) * KP + 16 * j2 + n] = gacc[p / NW][i];
              gacc[p / NW][i] = 0.f;
            }
    }
    if (!has_next) break;
    s = ns;
    cr = ncr;
    row0 = nrow0;
    nrows = nnrows;
    buf ^= 1;
  }
}

// ---------------------------------------------------------------------------
// Y = sum_i rho_i^-2 P_i (sum_{s in i} Z_s)   (Eq. 10), FP64.
// Grid: (column tiles of CT TRs) x (groups of gsub subjects).
// ---------------------------------------------------------------------------

template <int KP, int CT>
__global__ __launch_bounds__(256) void k_ereduce(RArgs a) {
  if (a.sc->status) return;
  // Thread t holds the RJ x CW block: features RJ (t / 16) + u, TRs
  // c0 + CW (t % 16) + m.
  constexpr int RJ = KP / 16, CW = CT / 16;
  __shared__ double Zs[KP][CT];
  __shared__ double Pt[KP][KP];  // P_i transposed: Pt[b][j] = P_i[j][b]
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * CT;
  const int rg = tid / 16, cg = tid % 16;
  double out[RJ][CW];
#pragma unroll
  for (int u = 0; u < RJ; ++u)
#pragma unroll
    for (int m = 0; m < CW; ++m) out[u][m] = 0.0;
  const int i0 = blockIdx.y * a.gsub;
  int i1 = i0 + a.gsub;
  if (i1 > a.N) i1 = a.N;
  for (int i = i0; i < i1; ++i) {
    const Subject su = a.subj[i];
    for (int idx = tid; idx < KP * CT; idx += 256) {
      const int j = idx / CT, cc = idx % CT;
      double s = 0.0;
      for (int sl = su.s_beg; sl < su.s_end; ++sl)
        s += (double)a.zpart[((int64_t)sl * KP + j) * a.ldt + c0 + cc];
      Zs[j][cc] = s;
    }
    const double* P = a.P64 + (int64_t)i * KP * KP;
    for (int idx = tid; idx < KP * KP; idx += 256) Pt[idx % KP][idx / KP] = P[idx];
    __syncthreads();
    const double w = 1.0 / a.rho2[i];
    double acc[RJ][CW];
#pragma unroll
    for (int u = 0; u < RJ; ++u)
#pragma unroll
      for (int m = 0; m < CW; ++m) acc[u][m] = 0.0;
#pragma unroll 4
    for (int b = 0; b < KP; ++b) {
      double pv[RJ], zv[CW];
#pragma unroll
      for (int u = 0; u < RJ; ++u) pv[u] = Pt[b][RJ * rg + u];
#pragma unroll
      for (int m = 0; m < CW; ++m) zv[m] = Zs[b][CW * cg + m];
#pragma unroll
      for (int u = 0; u < RJ; ++u)
#pragma unroll
        for (int m = 0; m < CW; ++m) acc[u][m] += pv[u] * zv[m];
    }
#pragma unroll
    for (int u = 0; u < RJ; ++u)
#pragma unroll
      for (int m = 0; m < CW; ++m) out[u][m] += w * acc[u][m];
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < RJ; ++u)
#pragma unroll
    for (int m = 0; m < CW; ++m)
      a.ygrp[((int64_t)blockIdx.y * KP + RJ * rg + u) * a.ldt + c0 + CW * cg + m] = out[u][m];
}

// ---------------------------------------------------------------------------
// Dense FP64 helpers for k x k matrices (one workgroup of NT threads),
// in place on one LDS matrix, row-major with leading dimension ld.
// ---------------------------------------------------------------------------
// In-place lower Cholesky (right-looking).  Returns false if not PD.
template <int NT>
__device__ bool chol_lower(double* A, int k, int ld, int* flag) {
  const int tid = threadIdx.x;
  if (tid == 0) *flag = 0;
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    if (tid == 0) {
      const double d = A[j * ld + j];
      if (!(d > 0.0)) {
        *flag = 1;
        A[j * ld + j] = 1.0;
      } else {
        A[j * ld + j] = sqrt(d);
      }
    }
    __syncthreads();
    const double djj = A[j * ld + j];
    for (int i = j + 1 + tid; i < k; i += NT) A[i * ld + j] /= djj;
    __syncthreads();
    const int m = k - 1 - j;
    for (int idx = tid; idx < m * m; idx += NT) {
      const int r = j + 1 + idx / m, c = j + 1 + idx % m;
      if (c <= r) A[r * ld + c] -= A[r * ld + j] * A[c * ld + j];
    }
    __syncthreads();
  }
  const bool ok = *flag == 0;
  __syncthreads();
  return ok;
}

// In place: the lower triangle of A (a Cholesky factor L) becomes X = L^-1.
// Forward elimination of L X = I, one pivot row per step with all rows below
// it updated in parallel.  While step m runs, row r of the storage holds X's
// columns c < m and L's columns c >= m.  Pivot row m is used unscaled
// (1 / L_mm folded into the update) and scaled one step later, when nothing
// reads it any more.  col: [k] doubles of scratch.
template <int NT>
__device__ void tri_inv_lower_inplace(double* A, int k, int ld, double* col) {
  const int tid = threadIdx.x;
  double prev_inv = 0.0;
  for (int m = 0; m < k; ++m) {
    const double inv = 1.0 / A[m * ld + m];
    for (int r = m + 1 + tid; r < k; r += NT) col[r] = A[r * ld + m];
    if (m > 0) {  // finish the previous pivot row
      for (int c = tid; c < m - 1; c += NT) A[(m - 1) * ld + c] *= prev_inv;
      if (tid == 0) A[(m - 1) * ld + m - 1] = prev_inv;
    }
    __syncthreads();
    const int w = m + 1;
    for (int idx = tid; idx < (k - 1 - m) * w; idx += NT) {
      const int r = m + 1 + idx / w, c = idx % w;
      const double l = col[r] * inv;
      if (c < m)
        A[r * ld + c] -= l * A[m * ld + c];
      else
        A[r * ld + m] = -l;
    }
    __syncthreads();
    prev_inv = inv;
  }
  if (k > 0) {
    for (int c = tid; c < k - 1; c += NT) A[(k - 1) * ld + c] *= prev_inv;
    if (tid == 0) A[(k - 1) * ld + k - 1] = prev_inv;
  }
  __syncthreads();
}

// In place: lower-triangular X (lower triangle of A) becomes the full
// symmetric X^T X.  Entries above the diagonal are formed first (that
// storage is free), the diagonal in diag[k], then mirrored down.
template <int NT>
__device__ void ltl_inplace(double* A, int k, int ld, double* diag) {
  const int tid = threadIdx.x;
  for (int idx = tid; idx < k * k; idx += NT) {
    const int a = idx / k, b = idx % k;
    if (a > b) continue;
    double s = 0.0;
    for (int m = b; m < k; ++m) s += A[m * ld + a] * A[m * ld + b];
    if (a == b)
      diag[a] = s;
    else
      A[a * ld + b] = s;
  }
  __syncthreads();
  for (int idx = tid; idx < k * k; idx += NT) {
    const int a = idx / k, b = idx % k;
    if (a > b)
      A[a * ld + b] = A[b * ld + a];
    else if (a == b)
      A[a * ld + a] = diag[a];
  }
  __syncthreads();
}

// out = X^T X for lower-triangular X (full symmetric result, row-major ldo).
template <int NT>
__device__ void ltl(const double* X, int k, int ld, double* out, int ldo) {
  for (int idx = threadIdx.x; idx < k * k; idx += NT) {
    const int a = idx / k, b = idx % k;
    const int m0 = a > b ? a : b;
    double s = 0.0;
    for (int m = m0; m < k; ++m) s += X[m * ld + a] * X[m * ld + b];
    out[a * ldo + b] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Posterior preparation (one workgroup): rho0 (Eq. 8), Cholesky of Sigma_s,
// Sigma_s^-1, M = (Sigma_s^-1 + rho0 I)^-1 (Eq. 7), log|I + rho0 Sigma_s| and
// the likelihood's data terms.  One k x k matrix in LDS (up to 132 KB at
// K padding 128); every factor and inverse is formed in place, by sixteen
// waves (the k sequential steps are short; more waves shorten each).
// ---------------------------------------------------------------------------

template <int KP>
__global__ __launch_bounds__(1024) void k_post_prep(PrepArgs a) {
  if (a.sc->status) return;
  constexpr int NT = 1024;
  constexpr int LD = KP + 1;
  __shared__ double A[KP * LD];
  __shared__ double vec[KP];
  __shared__ double red[NT / 64];
  __shared__ int flag;
  const int tid = threadIdx.x, k = a.k;

  double r0 = 0.0, vl = 0.0, cr = 0.0;
  for (int i = tid; i < a.N; i += NT) {
    const double r = a.rho2[i];
    r0 += 1.0 / r;
    vl += (double)a.subj[i].v * log(r);
    cr += a.c[i] / r;
  }
  const double rho0 = block_sum_nt<NT>(r0, red);
  const double svl = block_sum_nt<NT>(vl, red);
  const double scr = block_sum_nt<NT>(cr, red);

  for (int idx = tid; idx < k * k; idx += NT)
    A[(idx / k) * LD + idx % k] = a.sig[(idx / k) * KP + idx % k];
  __syncthreads();
  bool ok = chol_lower<NT>(A, k, LD, &flag);
  double ld1 = 0.0;
  for (int j = tid; j < k; j += NT) ld1 += 2.0 * log(A[j * LD + j]);
  ld1 = block_sum_nt<NT>(ld1, red);
  tri_inv_lower_inplace<NT>(A, k, LD, vec);
  ltl_inplace<NT>(A, k, LD, vec);  // A = Sigma_s^-1
  for (int j = tid; j < k; j += NT) A[j * LD + j] += rho0;
  __syncthreads();
  ok = chol_lower<NT>(A, k, LD, &flag) && ok;
  double ld2 = 0.0;
  for (int j = tid; j < k; j += NT) ld2 += 2.0 * log(A[j * LD + j]);
  ld2 = block_sum_nt<NT>(ld2, red);
  tri_inv_lower_inplace<NT>(A, k, LD, vec);
  for (int idx = tid; idx < KP * KP; idx += NT) a.M[idx] = 0.0;
  __syncthreads();
  ltl<NT>(A, k, LD, a.M, KP);
  if (tid == 0) {
    a.sc->rho0 = rho0;
    a.sc->sum_vlogrho = svl;
    a.sc->sum_c_rho = scr;
    a.sc->logdet = ld1 + ld2;  // log|Sigma_s| + log|Sigma_s^-1 + rho0 I|
    if (!ok && a.sc->status == 0) a.sc->status = 5;  // SRM_E_NOTPD
  }
}

// ---------------------------------------------------------------------------
// S = M Y on column tiles (Eq. 10), its records, S S^T and tr(Y^T S) partials.
// ---------------------------------------------------------------------------

template <int KP, int PREC>
__global__ __launch_bounds__(256) void k_post_s(SArgs a) {
  if (a.sc->status) return;
  constexpr int CT = 16;
  constexpr int NB = KP / 16;
  __shared__ double Ys[KP][CT];
  __shared__ double Ss[KP][CT];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * CT;
  for (int idx = tid; idx < KP * CT; idx += 256) {
    const int j = idx / CT, cc = idx % CT;
    double s = 0.0;
    for (int gq = 0; gq < a.ngrp; ++gq)
      s += a.ygrp[((int64_t)gq * KP + j) * a.ldt + c0 + cc];
    Ys[j][cc] = s;
  }
  __syncthreads();
  double tr = 0.0;
  for (int idx = tid; idx < KP * CT; idx += 256) {
    const int j = idx / CT, cc = idx % CT;
    const int64_t col = c0 + cc;
    double s = 0.0;
    if (j < a.k && col < a.t) {
      for (int b = 0; b < a.k; ++b) s += a.M[j * KP + b] * Ys[b][cc];
    }
    Ss[j][cc] = s;
    tr += s * Ys[j][cc];
    a.s64[(int64_t)j * a.ldt + col] = s;
    const int jb = j >> 4;
    if constexpr (PREC == P_FP32) {
      const int64_t tb = col >> 4;
      const int lane = (j & 15) + 16 * (int)((col & 15) >> 2);
      ((float*)a.sh)[((tb * NB + jb) * 64 + lane) * 4 + (col & 3)] = (float)s;
    } else {
      const int64_t tb = col >> 5;
      const int lane = (j & 15) + 16 * (int)((col & 31) >> 3);
      const int64_t o = ((tb * NB + jb) * 64 + lane) * 8 + (col & 7);
      const float f = (float)s;
      const uint32_t h = f2bf(f);
      ((uint16_t*)a.sh)[o] = (uint16_t)h;
      ((uint16_t*)a.sl)[o] = (uint16_t)f2bf(f - bf2f(h));
    }
  }
  tr = block_sum256(tr, red);
  if (tid == 0) a.trpart[blockIdx.x] = tr;
  for (int idx = tid; idx < KP * KP; idx += 256) {
    const int p = idx / KP, q = idx % KP;
    double s = 0.0;
#pragma unroll
    for (int cc = 0; cc < CT; ++cc) s += Ss[p][cc] * Ss[q][cc];
    a.sspart[(int64_t)blockIdx.x * KP * KP + idx] = s;
  }
}

// ---------------------------------------------------------------------------
// Sigma_s = M + S S^T / t (Eq. 11), tau = tr(Sigma_s), log-likelihood.
// ---------------------------------------------------------------------------

// Sigma_s_new = M + S S^T / t (Eq. 11), symmetrised: one entry per thread,
// the column-tile partials of S S^T summed in a fixed order.
template <int KP>
__global__ __launch_bounds__(256) void k_post_sig(FinArgs a) {
  if (a.sc->status) return;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= KP * KP) return;
  const int p = idx / KP, q = idx % KP;
  double v = 0.0;
  if (p < a.k && q < a.k) {
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < a.nblk; ++b) {
      s1 += a.sspart[(int64_t)b * KP * KP + p * KP + q];
      s2 += a.sspart[(int64_t)b * KP * KP + q * KP + p];
    }
    const double v1 = a.M[p * KP + q] + s1 / (double)a.t;
    const double v2 = a.M[q * KP + p] + s2 / (double)a.t;
    v = 0.5 * (v1 + v2);
  }
  a.sig_new[idx] = v;
}

// tr(Sigma_s_new) and the log-likelihood of the parameters entering the step.
template <int KP>
__global__ __launch_bounds__(256) void k_post_fin(FinArgs a) {
  if (a.sc->status) return;
  __shared__ double red[4];
  const int tid = threadIdx.x;
  double tau = 0.0;
  for (int p = tid; p < a.k; p += 256) tau += a.sig_new[p * KP + p];
  tau = block_sum256(tau, red);
  if (tid == 0) {
    double tr = 0.0;
    for (int b = 0; b < a.nblk; ++b) tr += a.trpart[b];
    const Scalars* s = a.sc;
    const double t = (double)a.t;
    const double ll = -0.5 * (t * a.Vtot * 1.8378770664093454836 +
                              t * s->sum_vlogrho + t * s->logdet +
                              s->sum_c_rho - tr);
    const int n = a.sc->ll_count;
    a.ll[n & (kLLCapacity - 1)] = ll;
    a.sc->ll_count = n + 1;
    a.sc->tau_new = tau;
  }
}

// Start of an iteration: the previous E-step's S, Sigma_s, tau become current.

__global__ __launch_bounds__(256) void k_copy_state(CopyArgs a) {
  if (a.sc->status) return;
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (int64_t i = i0; i < a.n_s64; i += stride) a.s64_cur[i] = a.s64_new[i];
  for (int64_t i = i0; i < a.n_srec16; i += stride) a.srec_cur[i] = a.srec_new[i];
  for (int64_t i = i0; i < a.n_sig; i += stride) a.sig_cur[i] = a.sig_new[i];
  if (i0 == 0) a.sc->tau_cur = a.sc->tau_new;
}

// ---------------------------------------------------------------------------
// Polar factor and rho update, one workgroup per subject (Eq. 4, reading of
// Eq. 5): G_i = sum_s G_s (FP64), cyclic Jacobi G_i = V diag(lambda) V^T,
// P_i = V diag(lambda^-1/2) V^T, tr(W_i^T A_i) = sum_j sqrt(lambda_j),
// rho_i^2 = (c_i - 2 tr(W_i^T A_i) + t tau) / (t v_i).
// ---------------------------------------------------------------------------

// C = A B for KP x KP FP64 matrices in LDS (row stride ld), zero padded
// beyond k: thread t holds the block rows t / 16 + 16 u, columns
// t % 16 + 16 v (256 threads).
template <int KP>
__device__ __forceinline__ void mm_blk(const double* A, const double* B, int ld, int k,
                                       double (&c)[KP / 16][KP / 16]) {
  constexpr int RB = KP / 16;
  const int rg = threadIdx.x / 16, cg = threadIdx.x % 16;
#pragma unroll
  for (int u = 0; u < RB; ++u)
#pragma unroll
    for (int v = 0; v < RB; ++v) c[u][v] = 0.0;
  for (int kk = 0; kk < k; ++kk) {
    double av[RB], bv[RB];
#pragma unroll
    for (int u = 0; u < RB; ++u) av[u] = A[(rg + 16 * u) * ld + kk];
#pragma unroll
    for (int v = 0; v < RB; ++v) bv[v] = B[kk * ld + cg + 16 * v];
#pragma unroll
    for (int u = 0; u < RB; ++u)
#pragma unroll
      for (int v = 0; v < RB; ++v) c[u][v] += av[u] * bv[v];
  }
}

__device__ double block_max256(double v, double* red /* >= 4 */) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  const double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return r;
}

// MODE: POLAR_BOTH runs the Newton-Schulz attempt and, if it is not taken,
// the Jacobi solver in one launch (K padding <= 80).  Above 80 the two are
// separate launches: POLAR_NS (256 threads) marks the subjects whose
// attempt was not taken in a.jac, and POLAR_JAC (1024 threads, G in LDS,
// V in global scratch) solves those.
enum { POLAR_BOTH = 0, POLAR_NS = 1, POLAR_JAC = 2 };

template <int KP, int NT, int MODE>
__global__ __launch_bounds__(NT) void k_polar(QArgs a) {
  // Workgroups of this launch raise the status themselves, so it is read
  // once per workgroup: every wave then takes the same early return.
  __shared__ int status_;
  if (threadIdx.x == 0) status_ = a.sc->status;
  __syncthreads();
  if (status_) return;
  constexpr int LD = KP + 1;
  // Three KP x KP buffers (G; V or the Newton-Schulz iterate X; a product
  // B) live in LDS for K padding <= 80, in global scratch above (except G
  // of the separate Jacobi launch, which is in LDS).  The Jacobi solver is
  // warm-started from stored eigenvectors up to 80 (its product passes go
  // through registers).
  constexpr bool WARM = KP <= 80;
  constexpr bool IN_LDS = KP <= 80;
  constexpr bool G_LDS = IN_LDS || MODE == POLAR_JAC;
  // Above 80, the Newton-Schulz launch keeps its iterate X in LDS (read by
  // every product of a step), G and B in global scratch.
  constexpr bool X_LDS = !IN_LDS && MODE == POLAR_NS;
  constexpr int MAXP = (KP + 1) / 2;
  constexpr int NE = (KP * KP + NT - 1) / NT;  // product entries per thread
  __shared__ double lds[IN_LDS ? 3 * KP * LD : (G_LDS || X_LDS ? KP * LD : 1)];
  __shared__ double cs_[MAXP], sn_[MAXP];
  __shared__ double red[4];
  __shared__ int pp_[MAXP], qq_[MAXP];
  __shared__ int rotated;
  __shared__ double isq[KP];  // lambda_j^-1/2
  const int i = blockIdx.x, tid = threadIdx.x, k = a.k;
  if constexpr (MODE == POLAR_JAC) {
    if (a.jac[i] == 0) return;  // whole workgroup: the Newton-Schulz step was taken
  }
  double* const gw = a.work + (int64_t)i * 3 * KP * LD;
  double* G = G_LDS ? lds : gw;
  double* V = IN_LDS ? G + KP * LD : gw + KP * LD;
  const Subject su = a.subj[i];
  const int m = (k + 1) & ~1;  // even player count; index k (if k odd) is a dummy
  const int npair = m / 2;

  // G_i from the slices' upper 16x16 tiles, mirrored; dummy row/col zero.
  for (int idx = tid; idx < m * m; idx += NT) {
    const int p = idx / m, q = idx % m;
    double s = 0.0;
    if (p < k && q < k) {
      const int r = p <= q ? p : q, cc = p <= q ? q : p;
      for (int sl = su.s_beg; sl < su.s_end; ++sl)
        s += (double)a.gpart[(int64_t)sl * KP * KP + r * KP + cc];
    }
    G[p * LD + q] = s;
  }
  const bool warm = WARM && a.sc->polar_warm != 0;
  {
    // P_i = G_i^{-1/2} by Newton-Schulz, then certified below.  From the
    // previous iteration's P_i: X <- X + X E / 2, E = I - X G X, quadratic
    // while the Gram changes little between iterations.  On the first
    // iteration, and where that start fails: the coupled form on Y = G / s, Z = I (s = |G|_F, so the
    // spectrum of Y lies in (0, 1]): T = (3 I - Z Y) / 2, Y <- Y T,
    // Z <- T Z, Z Y -> I and Z -> Y_0^{-1/2}, stable where the uncoupled form
    // from a scaled identity is not.  Taken when E vanishes to rounding and
    // |X|_F^2 |G|_F < 1e13, which certifies lambda_min > 1e-13 lambda_max;
    // otherwise the Jacobi eigensolver below decides.
    if (NT == 256) {
      constexpr int RB = KP / 16;
      double* X = X_LDS ? lds : G + KP * LD;
      double* B = G + 2 * KP * LD;
      const int rg = tid / 16, cg = tid % 16;
      double c[RB][RB];
      auto store = [&](double* M) {
#pragma unroll
        for (int u = 0; u < RB; ++u)
#pragma unroll
          for (int v = 0; v < RB; ++v) M[(rg + 16 * u) * LD + cg + 16 * v] = c[u][v];
      };
      // max |I - c| over the k x k entries of this thread's block
      auto dev_from_i = [&]() {
        double em = 0.0;
#pragma unroll
        for (int u = 0; u < RB; ++u)
#pragma unroll
          for (int v = 0; v < RB; ++v) {
            const int p = rg + 16 * u, q = cg + 16 * v;
            c[u][v] = (p < k && q < k) ? (p == q ? 1.0 : 0.0) - c[u][v] : 0.0;
            em = fmax(em, fabs(c[u][v]));
          }
        return em;
      };
      // Certifies X against G (emax = max |I - X G X|) and writes P_i;
      // false: not taken, G unchanged.
      auto certify = [&](double emax) {
        // |X|_F^2, |G|_F^2 and tr(G X) = sum of the singular values of A_i
        double nx = 0.0, ng = 0.0, tgx = 0.0;
        for (int idx = tid; idx < k * k; idx += NT) {
          const int p = idx / k, q = idx % k;
          const double x = X[p * LD + q], gv = G[p * LD + q];
          nx += x * x;
          ng += gv * gv;
          tgx += gv * X[q * LD + p];
        }
        nx = block_sum256(nx, red);
        ng = block_sum256(ng, red);
        tgx = block_sum256(tgx, red);
        if (emax <= 1e-12 && nx * sqrt(ng) < 1e13) {
          double* P = a.P64 + (int64_t)i * KP * KP;
          for (int idx = tid; idx < KP * KP; idx += NT) {
            const int p = idx / KP, q = idx % KP;
            P[idx] = (p < k && q < k) ? 0.5 * (X[p * LD + q] + X[q * LD + p]) : 0.0;
          }
          if constexpr (WARM) {
            // No eigenvectors yet: the identity is the (orthogonal) warm start
            // a later Jacobi solve of this subject rotates from.
            if (a.sc->polar_warm == 0) {
              double* Vp = a.vprev + (int64_t)i * KP * KP;
              for (int idx = tid; idx < m * m; idx += NT)
                Vp[(idx / m) * KP + idx % m] = (idx / m == idx % m && idx / m < k) ? 1.0 : 0.0;
            }
          }
          if (tid == 0) {
            const double t = (double)a.t;
            if (!a.init_mode) a.rho2[i] = (a.c[i] - 2.0 * tgx + t * a.sc->tau_cur) / (t * su.v);
            if (MODE == POLAR_NS) a.jac[i] = 0;
          }
          return true;
        }
        return false;
      };
      bool done = false;
      if (a.sc->polar_warm != 0) {
        double emax = 1.0;
        const double* Pp = a.P64 + (int64_t)i * KP * KP;
        for (int idx = tid; idx < KP * KP; idx += NT) {
          const int p = idx / KP, q = idx % KP;
          X[p * LD + q] = Pp[idx];
          if (p >= m || q >= m) G[p * LD + q] = 0.0;  // zero padding up to KP
        }
        __syncthreads();
        for (int it = 0; it < 8; ++it) {
          mm_blk<KP>(G, X, LD, k, c);  // T = G X
          __syncthreads();
#pragma unroll
          for (int u = 0; u < RB; ++u)
#pragma unroll
            for (int v = 0; v < RB; ++v) B[(rg + 16 * u) * LD + cg + 16 * v] = c[u][v];
          __syncthreads();
          mm_blk<KP>(X, B, LD, k, c);  // X G X
          double em = 0.0;
#pragma unroll
          for (int u = 0; u < RB; ++u)
#pragma unroll
            for (int v = 0; v < RB; ++v) {
              const int p = rg + 16 * u, q = cg + 16 * v;
              c[u][v] = (p < k && q < k) ? (p == q ? 1.0 : 0.0) - c[u][v] : 0.0;
              em = fmax(em, fabs(c[u][v]));
            }
          emax = block_max256(em, red);  // also orders the reads of B
#pragma unroll
          for (int u = 0; u < RB; ++u)
#pragma unroll
            for (int v = 0; v < RB; ++v) B[(rg + 16 * u) * LD + cg + 16 * v] = c[u][v];
          __syncthreads();
          if (emax <= 1e-14 || !(emax < 0.5)) break;
          mm_blk<KP>(X, B, LD, k, c);  // X E
          __syncthreads();
          // X <- X + (X E + E X) / 4: the symmetric part of X + X E / 2
#pragma unroll
          for (int u = 0; u < RB; ++u)
#pragma unroll
            for (int v = 0; v < RB; ++v) B[(rg + 16 * u) * LD + cg + 16 * v] = c[u][v];
          __syncthreads();
          for (int idx = tid; idx < KP * KP; idx += NT) {
            const int p = idx / KP, q = idx % KP;
            if (p < q) {
              const double d = 0.25 * (B[p * LD + q] + B[q * LD + p]);
              X[p * LD + q] += d;
              X[q * LD + p] += d;
            } else if (p == q) {
              X[p * LD + p] += 0.5 * B[p * LD + p];
            }
          }
          __syncthreads();
        }
        done = certify(emax);
      }
      if (!done) {  // first iteration, or the warm start failed
        double emax = 1.0;
        __syncthreads();  // G complete
        double g2 = 0.0;
        for (int idx = tid; idx < k * k; idx += NT) {
          const double gv = G[(idx / k) * LD + idx % k];
          g2 += gv * gv;
        }
        const double sc = sqrt(block_sum256(g2, red));
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        for (int idx = tid; idx < KP * KP; idx += NT) {
          const int p = idx / KP, q = idx % KP;
          const bool in = p < k && q < k;
          G[p * LD + q] = in ? G[p * LD + q] * inv : 0.0;  // Y_0 (and zero padding)
          X[p * LD + q] = (in && p == q) ? 1.0 : 0.0;      // Z_0
        }
        __syncthreads();
        double prev = 1e300;
        for (int it = 0; it < 64; ++it) {
          mm_blk<KP>(X, G, LD, k, c);  // Z Y
          const double em = dev_from_i();
          const double e = block_max256(em, red);  // also orders the reads of X, G
          if (e <= 1e-14 || !(e < 1.5) || (e < 1e-10 && e > 0.25 * prev)) break;
          prev = e;
          // T = (3 I - Z Y) / 2 = I + (I - Z Y) / 2
#pragma unroll
          for (int u = 0; u < RB; ++u)
#pragma unroll
            for (int v = 0; v < RB; ++v) {
              const int p = rg + 16 * u, q = cg + 16 * v;
              c[u][v] = (p < k && q < k) ? (p == q ? 1.0 : 0.0) + 0.5 * c[u][v] : 0.0;
            }
          store(B);
          __syncthreads();
          mm_blk<KP>(G, B, LD, k, c);  // Y T
          __syncthreads();
          store(G);
          mm_blk<KP>(B, X, LD, k, c);  // T Z
          __syncthreads();
          store(X);
          __syncthreads();
        }
        // X = Z / sqrt(s) = G^{-1/2}; G again from the slices (Y overwrote it)
        const double xs = sc > 0.0 ? 1.0 / sqrt(sc) : 0.0;
        for (int idx = tid; idx < KP * KP; idx += NT) {
          const int p = idx / KP, q = idx % KP;
          X[p * LD + q] *= xs;
          double gv = 0.0;
          if (p < k && q < k) {
            const int r = p <= q ? p : q, cc = p <= q ? q : p;
            for (int sl = su.s_beg; sl < su.s_end; ++sl)
              gv += (double)a.gpart[(int64_t)sl * KP * KP + r * KP + cc];
          }
          G[p * LD + q] = gv;
        }
        __syncthreads();
        mm_blk<KP>(G, X, LD, k, c);  // G X
        store(B);
        __syncthreads();
        mm_blk<KP>(X, B, LD, k, c);  // X G X
        emax = block_max256(dev_from_i(), red);
        done = certify(emax);
      }
      if (done) return;
      __syncthreads();  // not taken: G is unchanged; the eigensolver decides
    }
  }
  if constexpr (MODE == POLAR_NS) {
    if (tid == 0) a.jac[i] = 1;
    return;
  }
  if constexpr (WARM) {
    const double* Vp = a.vprev + (int64_t)i * KP * KP;
    for (int idx = tid; idx < m * m; idx += NT) {
      const int p = idx / m, q = idx % m;
      V[p * LD + q] = warm ? Vp[p * KP + q] : (p == q && p < k ? 1.0 : 0.0);
    }
    __syncthreads();
    if (warm) {  // G <- V^T (G V), then rotate further from V
      double tv[NE];
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int idx = tid + NT * u;
        double s = 0.0;
        if (idx < k * k) {
          const int p = idx / k, q = idx % k;
          for (int r = 0; r < k; ++r) s += G[p * LD + r] * V[r * LD + q];
        }
        tv[u] = s;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int idx = tid + NT * u;
        if (idx < k * k) G[(idx / k) * LD + idx % k] = tv[u];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int idx = tid + NT * u;
        double s = 0.0;
        if (idx < k * k) {
          const int p = idx / k, q = idx % k;
          for (int r = 0; r < k; ++r) s += V[r * LD + p] * G[r * LD + q];
        }
        tv[u] = s;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int idx = tid + NT * u;
        if (idx < k * k) G[(idx / k) * LD + idx % k] = tv[u];
      }
    }
  } else {
    for (int idx = tid; idx < m * m; idx += NT) {
      const int p = idx / m, q = idx % m;
      V[p * LD + q] = (p == q && p < k) ? 1.0 : 0.0;
    }
  }
  __syncthreads();

  // Cyclic Jacobi, round-robin (circle) ordering.  Each round's rotations
  // act on disjoint index pairs, so G <- J^T G J splits into independent
  // 2x2 blocks B_xy <- J_x^T B_xy J_y, and V <- V J into row pairs.
  for (int sweep = 0; sweep < 40; ++sweep) {
    // A sweep in which no pair passes the rotation test changes nothing:
    // test all pairs at once and stop before such a sweep.
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int idx = tid; idx < m * m; idx += NT) {
      const int p = idx / m, q = idx % m;
      if (p < q && q < k) {
        const double apq = G[p * LD + q];
        if (fabs(apq) > 1e-15 * sqrt(fabs(G[p * LD + p] * G[q * LD + q])) && apq != 0.0)
          rotated = 1;
      }
    }
    __syncthreads();
    if (!rotated) break;
    for (int rnd = 0; rnd < m - 1; ++rnd) {
      if (tid < npair) {
        int p, q;
        if (tid == 0) {
          p = m - 1;
          q = rnd;
        } else {
          p = (rnd + tid) % (m - 1);
          q = (rnd - tid + m - 1) % (m - 1);
        }
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        double c = 1.0, s = 0.0;
        if (q < k) {
          const double app = G[p * LD + p], aqq = G[q * LD + q];
          const double apq = G[p * LD + q];
          if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && apq != 0.0) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) /
                              (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        cs_[tid] = c;
        sn_[tid] = s;
        pp_[tid] = p;
        qq_[tid] = q;
      }
      __syncthreads();
      for (int idx = tid; idx < npair * npair; idx += NT) {
        const int x = idx / npair, y = idx % npair;
        const int p = pp_[x], q = qq_[x], r = pp_[y], t = qq_[y];
        const double cx = cs_[x], sx = sn_[x], cy = cs_[y], sy = sn_[y];
        const double b00 = G[p * LD + r], b01 = G[p * LD + t];
        const double b10 = G[q * LD + r], b11 = G[q * LD + t];
        const double m00 = cx * b00 - sx * b10, m01 = cx * b01 - sx * b11;
        const double m10 = sx * b00 + cx * b10, m11 = sx * b01 + cx * b11;
        G[p * LD + r] = cy * m00 - sy * m01;
        G[p * LD + t] = sy * m00 + cy * m01;
        G[q * LD + r] = cy * m10 - sy * m11;
        G[q * LD + t] = sy * m10 + cy * m11;
      }
      // V <- V J: all of a thread's loads first, then its stores (V may be
      // in global memory, where a load after each store would wait).
      {
        constexpr int NV = (MAXP * KP + NT - 1) / NT;
        double vp[NV], vq[NV];
#pragma unroll
        for (int u = 0; u < NV; ++u) {
          const int idx = tid + NT * u;
          if (idx < npair * m) {
            const int x = idx / m, j = idx % m;
            vp[u] = V[j * LD + pp_[x]];
            vq[u] = V[j * LD + qq_[x]];
          }
        }
#pragma unroll
        for (int u = 0; u < NV; ++u) {
          const int idx = tid + NT * u;
          if (idx < npair * m) {
            const int x = idx / m, j = idx % m;
            const double c = cs_[x], s = sn_[x];
            V[j * LD + pp_[x]] = c * vp[u] - s * vq[u];
            V[j * LD + qq_[x]] = s * vp[u] + c * vq[u];
          }
        }
      }
      __syncthreads();
    }
  }

  // Eigenvalues; rank check; sum of singular values of A_i.
  double lmax = 0.0, lmin = 1e300, ssq = 0.0;
  for (int j = 0; j < k; ++j) {
    const double l = G[j * LD + j];
    lmax = fmax(lmax, l);
    lmin = fmin(lmin, l);
  }
  const bool rank_ok = lmin > 1e-13 * lmax && lmax > 0.0;
  for (int j = 0; j < k; ++j) ssq += sqrt(fmax(G[j * LD + j], 0.0));
  for (int j = tid; j < k; j += NT) isq[j] = rank_ok ? 1.0 / sqrt(G[j * LD + j]) : 0.0;
  __syncthreads();
  // P = V diag(lambda^-1/2) V^T  (written zero padded to KP x KP)
  double* P = a.P64 + (int64_t)i * KP * KP;
  for (int idx = tid; idx < KP * KP; idx += NT) {
    const int p = idx / KP, q = idx % KP;
    double s = 0.0;
    if (p < k && q < k && rank_ok) {
      for (int j = 0; j < k; ++j) s += V[p * LD + j] * V[q * LD + j] * isq[j];
    }
    P[idx] = s;
  }
  if constexpr (WARM) {
    double* Vp = a.vprev + (int64_t)i * KP * KP;
    for (int idx = tid; idx < m * m; idx += NT) {
      const int p = idx / m, q = idx % m;
      Vp[p * KP + q] = V[p * LD + q];
    }
  }
  if (tid == 0) {
    const double t = (double)a.t;
    const double r = (a.c[i] - 2.0 * ssq + t * a.sc->tau_cur) / (t * su.v);
    if (!a.init_mode) a.rho2[i] = rank_ok ? r : 1.0;
    if (!rank_ok && a.sc->status == 0) a.sc->status = 4;  // SRM_E_RANK
  }
}

// Marks the stored eigenvectors as a valid warm start (after every subject's
// polar step of an iteration).
__global__ void k_polar_done(Scalars* sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && sc->status == 0) sc->polar_warm = 1;
}

// ---------------------------------------------------------------------------
// Results: W_i = A_i P_i (deferred polar factor) and the transform
// S_new = W_i^T (X_new - mu_i 1^T) = P_i A_i^T (X_new - mu_i 1^T).
// ---------------------------------------------------------------------------
template <int KP>
__device__ __forceinline__ double a_elem(const void* ah, const void* al,
                                         int prec, int64_t R, int b) {
  constexpr int NB = KP / 16;
  const int64_t rb = R >> 5;
  const int rr = (int)(R & 31);
  const int g = (rr & 15) >> 2, e = ((rr >> 4) << 2) + (rr & 3);
  const int lane = (b & 15) + 16 * g;
  const int64_t o = ((rb * NB + (b >> 4)) * 64 + lane) * 8 + e;
  if (prec == P_FP32) return (double)((const float*)ah)[o];
  return (double)bf2f(((const uint16_t*)ah)[o]) +
         (double)bf2f(((const uint16_t*)al)[o]);
}


template <int KP>
__global__ __launch_bounds__(256) void k_get_w(WArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)a.v * a.k) return;
  const int64_t r = idx / a.k;
  const int j = (int)(idx % a.k);
  double s = 0.0;
  for (int b = 0; b < a.k; ++b)
    s += a_elem<KP>(a.ah, a.al, a.prec, a.row0 + r, b) * a.P[b * KP + j];
  a.dst[idx] = (float)s;
}


// Partial Z[:, cols] = sum over a row split of A[r, :]^T (x_r - mu_r).
template <int KP>
__global__ __launch_bounds__(256) void k_transform_part(TArgs a) {
  constexpr int NJ = KP / 4;
  const int c = threadIdx.x & 63, jr = threadIdx.x >> 6;
  const int64_t col = (int64_t)blockIdx.x * 64 + c;
  const int r0 = blockIdx.y * a.rows_per_split;
  int r1 = r0 + a.rows_per_split;
  if (r1 > a.v) r1 = a.v;
  float acc[NJ];
#pragma unroll
  for (int u = 0; u < NJ; ++u) acc[u] = 0.f;
  if (col < a.tn) {
    for (int r = r0; r < r1; ++r) {
      const float x = (float)(((double)a.X[(int64_t)r * a.ldx + col] - a.mu[a.row0 + r]) *
                              a.isd[a.row0 + r]);
#pragma unroll
      for (int u = 0; u < NJ; ++u)
        acc[u] += (float)a_elem<KP>(a.ah, a.al, a.prec, a.row0 + r, jr + 4 * u) * x;
    }
#pragma unroll
    for (int u = 0; u < NJ; ++u)
      a.part[((int64_t)blockIdx.y * KP + jr + 4 * u) * a.tn + col] = acc[u];
  }
}


template <int KP>
__global__ __launch_bounds__(256) void k_transform_fin(TFArgs a) {
  __shared__ double Zs[KP][64];
  const int c = threadIdx.x & 63, jr = threadIdx.x >> 6;
  const int64_t col = (int64_t)blockIdx.x * 64 + c;
  for (int j = jr; j < KP; j += 4) {
    double s = 0.0;
    if (col < a.tn)
      for (int sp = 0; sp < a.nsplit; ++sp)
        s += (double)a.part[((int64_t)sp * KP + j) * a.tn + col];
    Zs[j][c] = s;
  }
  __syncthreads();
  if (col >= a.tn) return;
  for (int j = jr; j < a.k; j += 4) {
    double s = 0.0;
    for (int b = 0; b < a.k; ++b) s += a.P[j * KP + b] * Zs[b][c];
    a.out[(int64_t)j * a.ldo + col] = (float)s;
  }
}

// Subject-to-subject mapping, second half: Y[:, cols] = A_j (P_j S_new),
// with S_new = W_i^T (X_new - mu_i 1^T) already in `s` (k rows, stride ld).

template <int KP>
__global__ __launch_bounds__(256) void k_map(MapArgs a) {
  __shared__ float T[KP][64];  // P_j S_new for this block's 64 columns
  const int c = threadIdx.x & 63, jr = threadIdx.x >> 6;
  const int64_t col = (int64_t)blockIdx.x * 64 + c;
  for (int j = jr; j < KP; j += 4) {
    double s = 0.0;
    if (j < a.k && col < a.tn)
      for (int b = 0; b < a.k; ++b) s += a.P[j * KP + b] * (double)a.s[b * a.lds + col];
    T[j][c] = (float)s;
  }
  __syncthreads();
  if (col >= a.tn) return;
  for (int64_t r = (int64_t)blockIdx.y * 4 + jr; r < a.v; r += (int64_t)gridDim.y * 4) {
    float acc = 0.f;
    for (int b = 0; b < a.k; ++b)
      acc += (float)a_elem<KP>(a.ah, a.al, a.prec, a.row0 + r, b) * T[b][c];
    a.out[r * a.ldo + col] = acc;
  }
}

// ---------------------------------------------------------------------------
// Sample-space iteration (the voxel-to-sample change of complexity of the
// Discussion): with A_i = Xhat_i S^T,
//   A_i^T Xhat_i = S G_i   and   A_i^T A_i = S G_i S^T,   G_i = Xhat_i^T Xhat_i,
// so after one pass that forms G_i the iteration never reads Xhat again.
// ---------------------------------------------------------------------------

// G_i tile (64 x 64 TRs) for an upper tile pair (ta <= tb), mirrored below
// the diagonal; one workgroup per (subject, pair), the pairs of a subject
// placed on one XCD so that its rows are fetched into that L2 once.  The
// contraction over the subject's rows runs on matrix cores with FP32
// accumulation over 16 row blocks per wave, flushed into FP64 accumulators;
// the four waves take interleaved blocks and are summed in a fixed order.
//  FP32 storage: 16x16x4 FP32 products, 16-row blocks;
//  BF16 forms:   16x16x32 bf16 products on the stored planes (all four
//                hi/lo products for hi + lo storage), 32-row blocks read as
//                four TRs x eight rows per lane (the rows-as-K layout).
template <int PREC>
__global__ __launch_bounds__(256) void k_gram_build(GBArgs a) {
  __shared__ double L[64][65];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const int npairs = a.nt * (a.nt + 1) / 2;
  const int h = xcd_remap(blockIdx.x, gridDim.x);
  const int subj = h / npairs;
  int idx = h % npairs, ta = 0;
  while (idx >= a.nt - ta) {
    idx -= a.nt - ta;
    ++ta;
  }
  const int tb = ta + idx;
  const Subject su = a.subj[subj];
  const int64_t ca = 64 * (int64_t)ta, cb = 64 * (int64_t)tb;
  const int ldt = (int)a.ldt;
  double acc64[4][4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc64[u][v][e] = 0.0;

  if constexpr (PREC == P_FP32) {
    // acc64[mb][nb][e] holds G[ca + 16 mb + 4 g + e][cb + 16 nb + n]
    const float* X = (const float*)a.xh;
    const int nstep = su.vp / 16;
    for (int s0 = wave; s0 < nstep; s0 += 4 * 16) {
      f32x4 acc[4][4];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
      const int s1 = min(nstep, s0 + 4 * 16);
      for (int st = s0; st < s1; st += 4) {
        const int64_t r = su.row0 + 16 * (int64_t)st + 4 * g;
        float xa[4][4], xb[4][4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int mb = 0; mb < 4; ++mb) xa[mb][e] = X[(r + e) * ldt + ca + 16 * mb + n];
        if (ta != tb) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) xb[nb][e] = X[(r + e) * ldt + cb + 16 * nb + n];
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb) xb[nb][e] = xa[nb][e];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
              acc[mb][nb] = mfma_f32(xa[mb][e], xb[nb][e], acc[mb][nb]);
      }
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc64[mb][nb][e] += (double)acc[mb][nb][e];
    }
  } else {
    // Lane (n, g) loads, for rows 4 g + (e & 3) + 16 (e >> 2) of a 32-row
    // block, the TRs 4 n .. 4 n + 3 of a tile; operand q (TR 4 n + q) then
    // holds that column's eight rows.  acc64[qa][qb][r] holds
    // G[ca + 16 g + 4 r + qa][cb + 4 n + qb].
    constexpr bool X2 = PREC == P_BF16X2;
    const uint16_t* XH = (const uint16_t*)a.xh;
    const uint16_t* XL = (const uint16_t*)a.xl;
    const int vo = (4 * g * ldt + 4 * n) * 2;
    const bool diag = ta == tb;
    const int nblk = su.vp / 32;
    uint2 ra[2][2][8], rbv[2][2][8];  // [buffer][plane][e]
    auto load = [&](int buf, int b) __attribute__((always_inline)) {
      const int64_t r0 = su.row0 + 32 * (int64_t)b;
      const auto AH = make_rsrc(XH + r0 * ldt + ca, 32u * ldt * 2u);
      const auto AL = make_rsrc(XL + r0 * ldt + ca, 32u * ldt * 2u);
      const auto BH = make_rsrc(XH + r0 * ldt + cb, 32u * ldt * 2u);
      const auto BL = make_rsrc(XL + r0 * ldt + cb, 32u * ldt * 2u);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int so = ((e & 3) + 16 * (e >> 2)) * ldt * 2;
        ra[buf][0][e] = bload8(AH, vo, so);
        if constexpr (X2) ra[buf][1][e] = bload8(AL, vo, so);
        if (!diag) {
          rbv[buf][0][e] = bload8(BH, vo, so);
          if constexpr (X2) rbv[buf][1][e] = bload8(BL, vo, so);
        }
      }
    };
    auto repack = [&](const uint2 (&x)[8], int q) __attribute__((always_inline)) {
      uint4 o;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const uint32_t a0 = (q < 2) ? x[2 * d].x : x[2 * d].y;
        const uint32_t a1 = (q < 2) ? x[2 * d + 1].x : x[2 * d + 1].y;
        ((uint32_t*)&o)[d] = (q & 1) ? ((a0 >> 16) | (a1 & 0xffff0000u))
                                     : ((a0 & 0xffffu) | (a1 << 16));
      }
      return o;
    };
    f32x4 acc[4][4];
    auto compute = [&](int buf) __attribute__((always_inline)) {
      uint4 Ah[4], Al[4], Bh[4], Bl[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        Ah[q] = repack(ra[buf][0], q);
        if constexpr (X2) Al[q] = repack(ra[buf][1], q);
        if (!diag) {
          Bh[q] = repack(rbv[buf][0], q);
          if constexpr (X2) Bl[q] = repack(rbv[buf][1], q);
        } else {
          Bh[q] = Ah[q];
          if constexpr (X2) Bl[q] = Al[q];
        }
      }
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 4; ++qb) {
          acc[qa][qb] = mfma_bf16(Ah[qa], Bh[qb], acc[qa][qb]);
          if constexpr (X2) {
            acc[qa][qb] = mfma_bf16(Ah[qa], Bl[qb], acc[qa][qb]);
            acc[qa][qb] = mfma_bf16(Al[qa], Bh[qb], acc[qa][qb]);
            acc[qa][qb] = mfma_bf16(Al[qa], Bl[qb], acc[qa][qb]);
          }
        }
    };
    for (int b0 = wave; b0 < nblk; b0 += 4 * 16) {
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 4; ++qb) acc[qa][qb] = f32x4{0.f, 0.f, 0.f, 0.f};
      const int b1 = min(nblk, b0 + 4 * 16);
      load(0, b0);
      for (int b = b0; b < b1; b += 8) {
        if (b + 4 < b1) load(1, b + 4);
        compute(0);
        if (b + 4 >= b1) break;
        if (b + 8 < b1) load(0, b + 8);
        compute(1);
      }
#pragma unroll
      for (int qa = 0; qa < 4; ++qa)
#pragma unroll
        for (int qb = 0; qb < 4; ++qb)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[qa][qb][r] += (double)acc[qa][qb][r];
    }
  }
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int pr = (PREC == P_FP32) ? 16 * u + 4 * g + e : 16 * g + 4 * e + u;
            const int pc = (PREC == P_FP32) ? 16 * v + n : 4 * n + v;
            double& d = L[pr][pc];
            d = (w == 0 ? 0.0 : d) + acc64[u][v][e];
          }
    }
    __syncthreads();
  }
  const int64_t gbase = (int64_t)subj * a.ldt * a.ldt;
  const int c = threadIdx.x & 63;
  auto put = [&](int64_t o, double v) {
    if (a.G64) a.G64[gbase + o] = v;
    else a.G[gbase + o] = (float)v;
  };
  for (int p = threadIdx.x >> 6; p < 64; p += 4) put((ca + p) * a.ldt + cb + c, L[p][c]);
  if (ta != tb)
    for (int p = threadIdx.x >> 6; p < 64; p += 4) put((cb + p) * a.ldt + ca + c, L[c][p]);
}

// BF16 forms: Z_i[:, q-tile] = S G_i[:, q-tile] for one 64-TR tile (FP32
// matrix cores, FP32 G_i, S from the FP64 posterior rounded to FP32), stored
// in the subject's E-phase partial, and the tile's share of Z_i S^T (FP32
// products, FP64 out).
// Wave w owns TRs q0 + 16 w .. + 15 of the tile for all features.
template <int KP>
__global__ __launch_bounds__(256) void k_gram_z(GZArgs a) {
  if (a.sc->status) return;
  constexpr int NB = KP / 16;
  constexpr int PC = 64;        // TRs per staged S chunk
  constexpr int LS = PC + 4;    // padded row of the staged chunk
  __shared__ float Ss[KP][LS];  // S[:, p0 .. p0 + 63], later S[:, q-tile]
  __shared__ float Zt[KP][LS];  // the Z tile
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int n = lane & 15, g = lane >> 4;
  const int qt = blockIdx.x, i = blockIdx.y;
  const int64_t q0 = 64 * (int64_t)qt;
  // G_i is stored in full and symmetric: the lane's column q of G_i is read
  // as row q, four TRs per 16-byte load.
  const float* Gq = a.G + (int64_t)i * a.ldt * a.ldt + (q0 + 16 * wave + n) * a.ldt;
  f32x4 acc[NB];
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) acc[jb] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t p0 = 0; p0 < a.t; p0 += PC) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < KP * PC / 2; idx += 256) {  // two TRs per load
      const int j = idx / (PC / 2), pp = 2 * (idx % (PC / 2));
      double2 v = make_double2(0.0, 0.0);
      if (j < a.k) v = *(const double2*)&a.S[(int64_t)j * a.ldt + p0 + pp];
      Ss[j][pp] = p0 + pp < a.t ? (float)v.x : 0.f;
      Ss[j][pp + 1] = p0 + pp + 1 < a.t ? (float)v.y : 0.f;
    }
    __syncthreads();
    // K-step of 16 TRs: lane group g takes TRs 4 g .. 4 g + 3 (one per
    // product), for both operands alike.
#pragma unroll 2
    for (int ps = 0; ps < PC; ps += 16) {
      const float4 g4 = *(const float4*)(Gq + p0 + ps + 4 * g);  // < ldt: chunks end at ldt
      const float gv[4] = {g4.x, g4.y, g4.z, g4.w};
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
        const float4 sv = *(const float4*)&Ss[16 * jb + n][ps + 4 * g];
        acc[jb] = mfma_f32(sv.x, gv[0], acc[jb]);
        acc[jb] = mfma_f32(sv.y, gv[1], acc[jb]);
        acc[jb] = mfma_f32(sv.z, gv[2], acc[jb]);
        acc[jb] = mfma_f32(sv.w, gv[3], acc[jb]);
      }
    }
  }
  // lane holds Z[16 jb + 4 g + r][q0 + 16 wave + n]
  float* Z = a.zpart + (int64_t)i * KP * a.ldt + q0 + 16 * wave + n;
#pragma unroll
  for (int jb = 0; jb < NB; ++jb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Z[(int64_t)(16 * jb + 4 * g + r) * a.ldt] = acc[jb][r];
      Zt[16 * jb + 4 * g + r][16 * wave + n] = acc[jb][r];
    }
  __syncthreads();
  for (int idx = threadIdx.x; idx < KP * 64; idx += 256) {
    const int l = idx >> 6, c = idx & 63;
    Ss[l][c] = (l < a.k && q0 + c < a.t) ? (float)a.S[(int64_t)l * a.ldt + q0 + c] : 0.f;
  }
  __syncthreads();
  // Gram share over the tile's 64 TRs: block (j1, j2) of Z S^T, blocks
  // dealt round-robin to the waves; K-permuted as above.
  double* out = a.gz + ((int64_t)i * a.nq + qt) * KP * KP;
  for (int blk = wave; blk < NB * NB; blk += 4) {
    const int j1 = blk / NB, j2 = blk % NB;
    f32x4 c4 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ps = 0; ps < 64; ps += 16) {
      const float4 zv = *(const float4*)&Zt[16 * j1 + n][ps + 4 * g];
      const float4 sv = *(const float4*)&Ss[16 * j2 + n][ps + 4 * g];
      c4 = mfma_f32(zv.x, sv.x, c4);
      c4 = mfma_f32(zv.y, sv.y, c4);
      c4 = mfma_f32(zv.z, sv.z, c4);
      c4 = mfma_f32(zv.w, sv.w, c4);
    }
    // lane holds share[16 j1 + 4 g + r][16 j2 + n]
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(16 * j1 + 4 * g + r) * KP + 16 * j2 + n] = (double)c4[r];
  }
}

// FP32 storage: the same products from an FP64 G_i, in FP64 throughout (the
// polar factor is then as consistent with A = Xhat S^T as in the streamed
// sweep).  Thread t holds a (KP / 16) x 4 block: features t / 16 + 16 i,
// TRs 4 (t % 16) + m.
template <int KP>
__global__ __launch_bounds__(256) void k_gram_z64(GZArgs a) {
  if (a.sc->status) return;
  constexpr int NI = KP / 16;
  constexpr int PC = 32;  // TRs per staged chunk
  constexpr int SM1 = PC * 64 + KP * (PC + 1), SM2 = 2 * KP * 65;
  __shared__ double sm[SM1 > SM2 ? SM1 : SM2];
  const int cg = threadIdx.x & 15, rg = threadIdx.x >> 4;
  const int qt = blockIdx.x, i = blockIdx.y;
  const int64_t q0 = 64 * (int64_t)qt;
  const double* G = a.G64 + (int64_t)i * a.ldt * a.ldt;
  double acc[NI][4];
#pragma unroll
  for (int u = 0; u < NI; ++u)
#pragma unroll
    for (int m = 0; m < 4; ++m) acc[u][m] = 0.0;
  double (*Gs)[64] = reinterpret_cast<double (*)[64]>(sm);                  // [PC][64]
  double (*Ss)[PC + 1] = reinterpret_cast<double (*)[PC + 1]>(sm + PC * 64);  // [KP][PC+1]
  for (int64_t p0 = 0; p0 < a.t; p0 += PC) {
    for (int idx = threadIdx.x; idx < PC * 64; idx += 256) {
      const int pp = idx >> 6, c = idx & 63;
      Gs[pp][c] = G[(p0 + pp) * a.ldt + q0 + c];
    }
    for (int idx = threadIdx.x; idx < KP * PC; idx += 256) {
      const int j = idx / PC, pp = idx % PC;
      Ss[j][pp] = (j < a.k && p0 + pp < a.t) ? a.S[(int64_t)j * a.ldt + p0 + pp] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int pp = 0; pp < PC; ++pp) {
      double gv[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) gv[m] = Gs[pp][4 * cg + m];
#pragma unroll
      for (int u = 0; u < NI; ++u) {
        const double sv = Ss[rg + 16 * u][pp];
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[u][m] += sv * gv[m];
      }
    }
    __syncthreads();
  }
  float* Z = a.zpart + (int64_t)i * KP * a.ldt;
#pragma unroll
  for (int u = 0; u < NI; ++u)
    *(float4*)(Z + (int64_t)(rg + 16 * u) * a.ldt + q0 + 4 * cg) =
        make_float4((float)acc[u][0], (float)acc[u][1], (float)acc[u][2], (float)acc[u][3]);
  // Gram share: sum over this tile's 64 TRs of Z[j][q] S[l][q].
  double (*Zt)[65] = reinterpret_cast<double (*)[65]>(sm);
  double (*St)[65] = reinterpret_cast<double (*)[65]>(sm + KP * 65);
#pragma unroll
  for (int u = 0; u < NI; ++u)
#pragma unroll
    for (int m = 0; m < 4; ++m) Zt[rg + 16 * u][4 * cg + m] = acc[u][m];
  for (int idx = threadIdx.x; idx < KP * 64; idx += 256) {
    const int l = idx >> 6, c = idx & 63;
    St[l][c] = (l < a.k && q0 + c < a.t) ? a.S[(int64_t)l * a.ldt + q0 + c] : 0.0;
  }
  __syncthreads();
  double* out = a.gz + ((int64_t)i * a.nq + qt) * KP * KP;
  for (int idx = threadIdx.x; idx < KP * KP; idx += 256) {
    const int j = idx / KP, l = idx % KP;
    double s = 0.0;
#pragma unroll 8
    for (int cc = 0; cc < 64; ++cc) s += Zt[j][cc] * St[l][cc];
    out[idx] = s;
  }
}

// gpart[i] = sum over column tiles of the Gram shares (fixed order).
template <int KP>
__global__ __launch_bounds__(256) void k_gram_gsum(GSArgs a) {
  if (a.sc->status) return;
  const int i = blockIdx.x;
  for (int idx = threadIdx.x; idx < KP * KP; idx += 256) {
    double s = 0.0;
    for (int qt = 0; qt < a.nq; ++qt) s += a.gz[((int64_t)i * a.nq + qt) * KP * KP + idx];
    a.gpart[(int64_t)i * KP * KP + idx] = (float)s;
  }
}

// ---------------------------------------------------------------------------
// Launch wrappers (template dispatch on K padding and storage format).
// ---------------------------------------------------------------------------
#define SRM_KP_SWITCH(KPV, ...)                          \
  switch (KPV) {                                         \
    case 16: { constexpr int KP = 16; __VA_ARGS__; } break;  \
    case 32: { constexpr int KP = 32; __VA_ARGS__; } break;  \
    case 48: { constexpr int KP = 48; __VA_ARGS__; } break;  \
    case 64: { constexpr int KP = 64; __VA_ARGS__; } break;  \
    case 80: { constexpr int KP = 80; __VA_ARGS__; } break;  \
    case 96: { constexpr int KP = 96; __VA_ARGS__; } break;  \
    case 112: { constexpr int KP = 112; __VA_ARGS__; } break; \
    case 128: { constexpr int KP = 128; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                \
  }

#define SRM_PREC_SWITCH(PV, ...)                                  \
  switch (PV) {                                                   \
    case P_FP32: { constexpr int PR = P_FP32; __VA_ARGS__; } break;   \
    case P_BF16: { constexpr int PR = P_BF16; __VA_ARGS__; } break;   \
    case P_BF16X2: { constexpr int PR = P_BF16X2; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;                         \
  }

hipError_t launch_convert(hipStream_t st, int grid, const ConvertArgs& a) {
  hipLaunchKernelGGL(k_convert, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_rowsum(hipStream_t st, int N, const double* rowc,
                         const Subject* subj, double* c) {
  hipLaunchKernelGGL(k_rowsum, dim3(N), dim3(256), 0, st, rowc, subj, c);
  return hipGetLastError();
}
hipError_t launch_mphase(hipStream_t st, int kp, int prec, int grid,
                         const MArgs& a) {
  SRM_KP_SWITCH(kp, SRM_PREC_SWITCH(prec,
      if constexpr (PR == P_FP32)
        hipLaunchKernelGGL((k_mphase<KP, PR>), dim3(grid), dim3(256), 0, st, a);
      else
        hipLaunchKernelGGL((k_mphase_s<KP, PR>), dim3(grid), dim3(256), 0, st, a)));
  return hipGetLastError();
}
hipError_t launch_ephase(hipStream_t st, int kp, int prec, int grid,
                         const EArgs& a) {
  SRM_KP_SWITCH(kp, SRM_PREC_SWITCH(prec,
      if constexpr (PR == P_FP32)
        hipLaunchKernelGGL((k_ephase<KP, PR>), dim3(grid), dim3(256), 0, st, a);
      else
        hipLaunchKernelGGL((k_ephase_s<KP, PR>), dim3(grid), dim3(512), 0, st, a)));
  return hipGetLastError();
}
int ephase_panel(int prec) { return prec == P_FP32 ? 256 : kEphasePanel; }
// TRs per k_ereduce column tile: the widest whose Z tile and P_i fit LDS
// together (FP64: KP x CT + KP x KP), so each P_i is staged by fewer
// workgroups.
int ereduce_ct(int kp) { return kp <= 112 ? 64 : 32; }
hipError_t launch_ereduce(hipStream_t st, int kp, int ncol, int ngrp,
                          const RArgs& a) {
  dim3 grid(ncol, ngrp);
  switch (ereduce_ct(kp)) {
    case 64: SRM_KP_SWITCH(kp, if constexpr (KP <= 112) hipLaunchKernelGGL(
                 (k_ereduce<KP, 64>), grid, dim3(256), 0, st, a)); break;
    default: SRM_KP_SWITCH(kp, if constexpr (KP > 112) hipLaunchKernelGGL(
                 (k_ereduce<KP, 32>), grid, dim3(256), 0, st, a)); break;
  }
  return hipGetLastError();
}
hipError_t launch_post_prep(hipStream_t st, int kp, const PrepArgs& a) {
  SRM_KP_SWITCH(kp, hipLaunchKernelGGL((k_post_prep<KP>), dim3(1), dim3(1024), 0, st, a));
  return hipGetLastError();
}
hipError_t launch_post_s(hipStream_t st, int kp, int prec, int nblk,
                         const SArgs& a) {
  SRM_KP_SWITCH(kp, SRM_PREC_SWITCH(prec,
      hipLaunchKernelGGL((k_post_s<KP, PR>), dim3(nblk), dim3(256), 0, st, a)));
  return hipGetLastError();
}
hipError_t launch_post_fin(hipStream_t st, int kp, const FinArgs& a) {
  SRM_KP_SWITCH(kp,
      hipLaunchKernelGGL((k_post_sig<KP>), dim3((KP * KP + 255) / 256), dim3(256), 0, st, a);
      hipLaunchKernelGGL((k_post_fin<KP>), dim3(1), dim3(256), 0, st, a));
  return hipGetLastError();
}
hipError_t launch_copy_state(hipStream_t st, const CopyArgs& a) {
  hipLaunchKernelGGL(k_copy_state, dim3(64), dim3(256), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_seed(hipStream_t st, int kp, const SeedArgs& a) {
  const int64_t n = (int64_t)a.vp * kp;
  const int grid = (int)((n + 255) / 256);
  SRM_KP_SWITCH(kp, hipLaunchKernelGGL((k_seed_a<KP>), dim3(grid), dim3(256), 0, st, a));
  return hipGetLastError();
}
hipError_t launch_polar(hipStream_t st, int kp, int N, const QArgs& a) {
  // Four waves per subject (one wave per subject measured 2x slower).  Above
  // K padding 80 the Jacobi fallback runs as its own launch of 16 waves per
  // subject, with G in LDS.
  SRM_KP_SWITCH(kp, if constexpr (KP <= 80) {
    hipLaunchKernelGGL((k_polar<KP, 256, POLAR_BOTH>), dim3(N), dim3(256), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_polar<KP, 256, POLAR_NS>), dim3(N), dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_polar<KP, 1024, POLAR_JAC>), dim3(N), dim3(1024), 0, st, a);
  });
  // The polar factor of a drawn start is no warm start for the first
  // iteration's Gram: the stored eigenvectors stay unused.
  if (!a.init_mode) hipLaunchKernelGGL(k_polar_done, dim3(1), dim3(64), 0, st, a.sc);
  return hipGetLastError();
}
hipError_t launch_get_w(hipStream_t st, int kp, const WArgs& a) {
  const int64_t n = (int64_t)a.v * a.k;
  const int grid = (int)((n + 255) / 256);
  SRM_KP_SWITCH(kp, hipLaunchKernelGGL((k_get_w<KP>), dim3(grid), dim3(256), 0, st, a));
  return hipGetLastError();
}
hipError_t launch_transform(hipStream_t st, int kp, int nsplit, const TArgs& a,
                            const TFArgs& f) {
  const int ncol = (int)((a.tn + 63) / 64);
  SRM_KP_SWITCH(kp,
      hipLaunchKernelGGL((k_transform_part<KP>), dim3(ncol, nsplit), dim3(256), 0, st, a);
      hipLaunchKernelGGL((k_transform_fin<KP>), dim3(ncol), dim3(256), 0, st, f));
  return hipGetLastError();
}

bool fused_supported(int kp, int prec, int64_t ldt) {
  return prec != P_FP32 && kp <= 64 && ldt <= 512 && ldt % 128 == 0;
}
// Chunk rows the register-ring sweep supports for ldt (16 ldt / 64, and 64
// with eight waves).
bool fused_chunk_ok(int64_t ldt, int chunk) {
  const int nw = (int)(ldt / 64);
  return chunk == 16 * nw || (nw == 8 && chunk == 64);
}
hipError_t launch_fused(hipStream_t st, int kp, int prec, int64_t ldt, int grid, int chunk,
                        const FusedArgs& a) {
  const int nw = (int)(ldt / 64);
  if (!fused_chunk_ok(ldt, chunk)) return hipErrorInvalidValue;
#define SRM_FUSED_LAUNCH(NWV, CHV)                                                \
    SRM_KP_SWITCH(kp, if constexpr (KP <= 64) {                                   \
      if (prec == P_BF16)                                                         \
        hipLaunchKernelGGL((k_fused<KP, P_BF16, NWV, CHV>), dim3(grid), dim3(NWV * 64), 0, \
                           st, a);                                                \
      else                                                                        \
        hipLaunchKernelGGL((k_fused<KP, P_BF16X2, NWV, CHV>), dim3(grid), dim3(NWV * 64), 0, \
                           st, a);                                                \
    });
  switch (nw) {
    case 2: SRM_FUSED_LAUNCH(2, 32) break;
    case 4: SRM_FUSED_LAUNCH(4, 64) break;
    case 6: SRM_FUSED_LAUNCH(6, 96) break;
    case 8:
      if (chunk == 64) { SRM_FUSED_LAUNCH(8, 64) } else { SRM_FUSED_LAUNCH(8, 128) }
      break;
    default: return hipErrorInvalidValue;
  }
#undef SRM_FUSED_LAUNCH
  return hipGetLastError();
}

// LDS bytes of k_staged<KP, PREC, NW> (0 when its wave split does not
// apply): two chunk buffers of PL x 2 x 2 NW records and TP x 2 NB slots.
constexpr int staged_lds(int kp, int prec, int nw) {
  const int nb = kp / 16, fpw = (nb % 2 == 0) ? 2 : nb, nfg = nb / fpw;
  if (nb < 1 || nw % nfg != 0) return 0;
  const int pl = prec == P_BF16X2 ? 2 : 1;
  return (2 * pl * 2 * 2 * nw + (nw / nfg) * 2 * nb) * 1024;
}
bool staged_supported(int kp, int prec, int64_t ldt) {
  const int nw = (int)(ldt / 64);
  const int lds = staged_lds(kp, prec, nw);
  return fused_supported(kp, prec, ldt) && lds > 0 && lds <= 160 * 1024;
}
hipError_t launch_staged(hipStream_t st, int kp, int prec, int64_t ldt, int grid,
                         const FusedArgs& a) {
  const int nw = (int)(ldt / 64);
#define SRM_STAGED_NW(NWV)                                                       \
  case NWV:                                                                     \
    SRM_KP_SWITCH(kp, if constexpr (KP <= 64) {                                 \
      if constexpr (staged_lds(KP, P_BF16, NWV) > 0 &&                          \
                    staged_lds(KP, P_BF16, NWV) <= 160 * 1024)                  \
        if (prec == P_BF16) {                                                   \
          hipLaunchKernelGGL((k_staged<KP, P_BF16, NWV>), dim3(grid), dim3(NWV * 64), 0, st, a); \
          break;                                                                \
        }                                                                       \
      if constexpr (staged_lds(KP, P_BF16X2, NWV) > 0 &&                        \
                    staged_lds(KP, P_BF16X2, NWV) <= 160 * 1024)                \
        if (prec == P_BF16X2) {                                                 \
          hipLaunchKernelGGL((k_staged<KP, P_BF16X2, NWV>), dim3(grid), dim3(NWV * 64), 0, st, a); \
          break;                                                                \
        }                                                                       \
      return hipErrorInvalidValue;                                              \
    } else { return hipErrorInvalidValue; });                                   \
    break;
  switch (nw) {
    SRM_STAGED_NW(2) SRM_STAGED_NW(4) SRM_STAGED_NW(6) SRM_STAGED_NW(8)
    default: return hipErrorInvalidValue;
  }
#undef SRM_STAGED_NW
  return hipGetLastError();
}

hipError_t launch_gram_build(hipStream_t st, int prec, int npairs, int N, const GBArgs& a) {
  const int grid = npairs * N;  // bounded by the planner
  SRM_PREC_SWITCH(prec, hipLaunchKernelGGL((k_gram_build<PR>), dim3(grid), dim3(256), 0,
                                           st, a));
  return hipGetLastError();
}

hipError_t launch_gram_iter(hipStream_t st, int kp, int N, const GZArgs& z, const GSArgs& g) {
  SRM_KP_SWITCH(kp,
      if (z.G64)
        hipLaunchKernelGGL((k_gram_z64<KP>), dim3(z.nq, N), dim3(256), 0, st, z);
      else
        hipLaunchKernelGGL((k_gram_z<KP>), dim3(z.nq, N), dim3(256), 0, st, z);
      hipLaunchKernelGGL((k_gram_gsum<KP>), dim3(N), dim3(256), 0, st, g));
  return hipGetLastError();
}

hipError_t launch_map(hipStream_t st, int kp, const MapArgs& a) {
  const int ncol = (int)((a.tn + 63) / 64);
  const int nrow = (int)std::min<int64_t>(1024, (a.v + 3) / 4);
  SRM_KP_SWITCH(kp, hipLaunchKernelGGL((k_map<KP>), dim3(ncol, nrow), dim3(256), 0, st, a));
  return hipGetLastError();
}

hipError_t occupancy_mphase(int kp, int prec, int* blocks) {
  SRM_KP_SWITCH(kp, SRM_PREC_SWITCH(prec,
      if constexpr (PR == P_FP32)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void*)k_mphase<KP, PR>, 256, 0);
      else
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void*)k_mphase_s<KP, PR>, 256, 0)));
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Static scratch of the no-allocation transform (srm_transform_static): the
// per-row-split partials of W_i^T (X_new - mu_i) live in this file-scope
// array instead of the context's workspace.  Each device holds its own copy;
// host code uses only the address hipGetSymbolAddress returns for it, looked
// up once per device at context set-up, never the array's name.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) float scratch[kStaticScratchBytes / sizeof(float)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

size_t static_scratch_bytes() { return kStaticScratchBytes; }

// Looks up this device's copy of `scratch` once (the device must be current).
hipError_t static_scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[dev] = ptr;
  return hipSuccess;
}

// The device address of `scratch` on device dev, or null before its set-up.
void* static_scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}

}  // namespace srm
