// The orthonormal DCT-II along x as a dense matrix product on the matrix cores of gfx950: the
// alternative to the radix transform passes for the sine/cosine transforms of the FFT-based
// Poisson solver (Sec. 4.2, item ii), kept as a measured variant (the evaluation uses the radix
// passes).
//
// For a tile of P consecutive z-pencils at fixed y, Y = C X with C the N x N DCT-II matrix
// (C[k][x] = s_k cos(pi k (2x + 1) / 2N), s_0 = sqrt(1/N), s_k = sqrt(2/N)) and X the N x P tile.
// float32 operands are split into bf16 pairs, v = hi + lo (both round-to-nearest-even), and the
// product is formed as Ch Xh + Ch Xl + Cl Xh with float32 accumulation (v_mfma_f32_32x32x16_bf16;
// the dropped Cl Xl term is 2^-16 of the product).  C comes pre-split in the A-operand order of
// the instruction (one contiguous 1 KiB load per wavefront and k-block, L2-resident); the tile is
// staged in LDS as hi and lo bf16 rows of pencils (x contiguous) and read as B operands.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "kernels.h"

namespace kfbi {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {

__device__ __forceinline__ uint32_t bf16_bits(float v) {  // round to nearest even (finite v)
  uint32_t u = __float_as_uint(v);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

template <int N, int P>
struct GemmCfg {
  static constexpr int RS = N + 8;          // staged row stride (bf16): rows stay 16-byte aligned
  static constexpr int RB = N / 32 / 4;     // 32-row output blocks per wavefront (4 wavefronts)
  static constexpr int CB = P / 32;         // 32-column output blocks
  static constexpr size_t BYTES = 2ull * P * RS * sizeof(uint16_t);
  static_assert(RB >= 1 && CB >= 1, "tile of at least 128 rows and 32 pencils");
};

// Cf[h][rb][kb][lane] (bf16x8): h = 0 hi, 1 lo; the A operand of output row block rb and k
// block kb: lane holds C[32 rb + lane % 32][16 kb + 8 (lane / 32) + i], i < 8.
template <int N, int P>
__global__ __launch_bounds__(256) void k_gemm_x(const float* __restrict__ in, float* __restrict__ out,
                                               const bf16x8* __restrict__ Cf) {
  extern __shared__ __align__(16) unsigned char smem[];
  using G = GemmCfg<N, P>;
  constexpr int RS = G::RS, RB = G::RB, CB = G::CB;
  uint16_t* Xs = reinterpret_cast<uint16_t*>(smem);  // [hi/lo][P][RS]
  constexpr int NTZ = N / P;
  const int y = blockIdx.x / NTZ, z0 = (blockIdx.x % NTZ) * P;
  const int64_t NN = (int64_t)N * N;
  const float* src = in + (int64_t)y * N + z0;
  // staging: items of 2 x-rows by 4 consecutive pencils (two 16-byte loads, four 4-byte LDS
  // stores per half)
  constexpr int ITEMS = (N / 2) * (P / 4);
  for (int e = threadIdx.x; e < ITEMS; e += 256) {
    const int x = 2 * (e / (P / 4)), p = 4 * (e % (P / 4));
    const float4 v0 = *reinterpret_cast<const float4*>(src + x * NN + p);
    const float4 v1 = *reinterpret_cast<const float4*>(src + (x + 1) * NN + p);
    const float a[4] = {v0.x, v0.y, v0.z, v0.w}, b[4] = {v1.x, v1.y, v1.z, v1.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t h0 = bf16_bits(a[c]), h1 = bf16_bits(b[c]);
      const uint32_t l0 = bf16_bits(a[c] - bf16_value(h0)), l1 = bf16_bits(b[c] - bf16_value(h1));
      *reinterpret_cast<uint32_t*>(Xs + (p + c) * RS + x) = h0 | (h1 << 16);
      *reinterpret_cast<uint32_t*>(Xs + (P + p + c) * RS + x) = l0 | (l1 << 16);
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  f32x16 acc[RB][CB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < CB; ++j) acc[i][j] = f32x16{};
  const uint16_t* bsrc = Xs + (lane % 32) * RS + 8 * (lane / 32);
  for (int kb = 0; kb < N / 16; ++kb) {
    bf16x8 bh[CB], bl[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      bh[cb] = *reinterpret_cast<const bf16x8*>(bsrc + (32 * cb) * RS + 16 * kb);
      bl[cb] = *reinterpret_cast<const bf16x8*>(bsrc + (P + 32 * cb) * RS + 16 * kb);
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int rb = wv * RB + i;
      const bf16x8 ah = Cf[((0 * (N / 32) + rb) * (N / 16) + kb) * 64 + lane];
      const bf16x8 al = Cf[((1 * (N / 32) + rb) * (N / 16) + kb) * 64 + lane];
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        acc[i][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[cb], acc[i][cb], 0, 0, 0);
        acc[i][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[cb], acc[i][cb], 0, 0, 0);
        acc[i][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[cb], acc[i][cb], 0, 0, 0);
      }
    }
  }
  // result register j of a lane: row 32 rb + 8 (j / 4) + 4 (lane / 32) + j % 4, column lane % 32
  float* dst = out + (int64_t)y * N + z0 + (lane % 32);
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int k = 32 * (wv * RB + i) + 8 * (j / 4) + 4 * (lane / 32) + (j % 4);
        dst[k * NN + 32 * cb] = acc[i][cb][j];
      }
}

template <int N, int P>
hipError_t gemm_n(const float* in, float* out, const void* Cf, hipStream_t s) {
  using G = GemmCfg<N, P>;
  if (G::BYTES > 65536)
    (void)hipFuncSetAttribute((const void*)k_gemm_x<N, P>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G::BYTES);
  hipLaunchKernelGGL((k_gemm_x<N, P>), dim3(N * (N / P)), dim3(256), G::BYTES, s, in, out,
                     static_cast<const bf16x8*>(Cf));
  return hipGetLastError();
}

uint16_t host_bf16(float v) {
  uint32_t u;
  std::memcpy(&u, &v, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float host_bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float v;
  std::memcpy(&v, &u, 4);
  return v;
}

}  // namespace

bool gemm_pass_supported(int N) { return N == 128 || N == 256 || N == 512; }

std::vector<uint16_t> gemm_dct2_fragments(int N) {
  std::vector<uint16_t> f(2ull * N * N);
  const int R = N / 32, Kb = N / 16;
  for (int rb = 0; rb < R; ++rb)
    for (int kb = 0; kb < Kb; ++kb)
      for (int lane = 0; lane < 64; ++lane)
        for (int i = 0; i < 8; ++i) {
          const int k = 32 * rb + lane % 32, x = 16 * kb + 8 * (lane / 32) + i;
          const double sk = (k == 0) ? std::sqrt(1.0 / N) : std::sqrt(2.0 / N);
          const float c = (float)(sk * std::cos(M_PI * k * (2.0 * x + 1.0) / (2.0 * N)));
          const uint16_t hi = host_bf16(c), lo = host_bf16(c - host_bf16_value(hi));
          const size_t o = (((size_t)rb * Kb + kb) * 64 + lane) * 8 + i;
          f[o] = hi;
          f[(size_t)N * N + o] = lo;
        }
  return f;
}

hipError_t launch_gemm_dct2_x(int N, const float* in, float* out, const void* Cf, hipStream_t s) {
  switch (N) {
    case 128: return gemm_n<128, 64>(in, out, Cf, s);
    case 256: return gemm_n<256, 64>(in, out, Cf, s);
    case 512: return gemm_n<512, 32>(in, out, Cf, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace kfbi
