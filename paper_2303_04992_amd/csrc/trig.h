// Pencil sine/cosine transforms in LDS for gfx950.
//
// The FFT-based Poisson solver of the paper (Sec. 4.2, items ii-iii) needs, per axis, the
// orthonormal DCT-II / DST-II (length N, cell-centred and tangential face axes), their
// inverses DCT-III / DST-III, and the DST-I (length N-1, the face-normal axis).  Here every
// transform of two real pencils is one complex FFT: for the DCT/DST pair the real pencils
// are reordered (even samples ascending, odd samples descending) so that a length-N complex
// FFT plus one twiddle per output gives the cosine sums (Makhoul's algorithm); DST-II is the
// DCT-II of the sign-alternated pencil read backwards; DST-I is the FFT of the odd extension
// of length 2N.
//
// The complex FFT of length L = R1 * M is done in register passes: each thread loads R1
// strided samples, does an R1-point DFT in registers and applies the L-point twiddles, the
// results are transposed through LDS (rows padded so the transposed reads hit distinct
// banks), and the M-point DFTs follow: one register pass (M = R2), or, for L = 512 at N = 512,
// two (M = R2 * R3 = 8 * 8, with the M-point twiddles between them and a second transpose),
// which keeps eight samples per task so that 512 threads hold a tile with 16 complex values
// each.  Small DFTs are unrolled radix-4/2 butterflies with literal twiddles.
//
// A workgroup owns a tile of W real pencils (W*sizeof(T) = 128 bytes, so every row of the
// tile along the contiguous z axis is one 128-byte segment), stored in LDS as rows of length
// N + 1.
#pragma once
#include <hip/hip_runtime.h>

namespace kfbi {

enum Kind { DCT2 = 0, DST2 = 1, DCT3 = 2, DST3 = 3, DST1 = 4 };

template <typename T>
struct C2 {
  T x, y;
};

template <typename T>
struct Tab {
  const C2<T>* tw;   // e^{-2 pi i k / N}, k < N
  const C2<T>* tw2;  // e^{-2 pi i k / 2N}, k < 2N
  const C2<T>* mk;   // e^{-i pi k / 2N}, k < N
  const T* sc;       // orthonormal DCT-II scale s_k: sqrt(1/N) (k=0), sqrt(2/N)
  const T* isc;      // 1 / s_k
  T s0, s1;          // s_0 and s_k (k > 0), the two values of sc, read without a table access
  T is0, is1;        // 1 / s_0 and 1 / s_k (k > 0)
  const T* sg2;      // sigma_k^2 = (4/h^2) sin^2(pi k / 2N), k < N   (DCT-II / DST-I modes)
  const T* sg2s;     // sigma_{k+1}^2, k < N                           (DST-II modes)
};

template <typename T>
__host__ __device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__host__ __device__ constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Tile configuration of one transform kind at grid size N.
template <typename T, int N, int KIND>
struct TileCfg {
  static constexpr int W = (int)(128 / sizeof(T)) < N ? (int)(128 / sizeof(T)) : N;  // pencils
  static constexpr int RS = N + 1;                                                  // row stride
  static constexpr int L = (KIND == DST1) ? 2 * N : N;                              // FFT length
  static constexpr int NJ = W / 2;                                                  // complex jobs
  static constexpr bool THREE = N >= 512 && L == 512;                                // three passes
  static constexpr int R1 = THREE ? 8 : 1 << ((ilog2(L) + 1) / 2);                  // first radix
  static constexpr int M = L / R1;                                  // length of the second stage
  static constexpr int R2 = THREE ? 8 : M;                                          // second radix
  static constexpr int R3 = M / R2;                                        // third radix (or 1)
#ifndef KFBI_LDS_PAD
#define KFBI_LDS_PAD 1, 1, 1
#endif
  // Row, transpose-job and spectrum-job padding.  LDS serves 8-byte accesses 16 lanes at a time
  // over 32 four-byte banks, and the 16 lanes of a group are the NJ = 16 jobs of a tile at the
  // same position (8 jobs of 16 bytes in float64): odd job strides put them in distinct banks.
  static constexpr int PAD[3] = {KFBI_LDS_PAD};
  static constexpr int P2 = M + PAD[0];                                              // padded row
  static constexpr int YS = R1 * P2 + PAD[1];                // job stride of the transpose buffer
  // second transpose (three passes): rows of R3 unpadded (the lanes of a 16-lane group differ
  // in the job only, both when it is written and when it is read), odd job stride
  static constexpr int P3 = R3;
  static constexpr int YS3 = R1 * R2 * P3 + PAD[1];
  static constexpr int ZS = L + PAD[2];                      // job stride of the spectra
  static constexpr int NT_CAP = N >= 512 ? 512 : 256;
  static constexpr int NT = (NJ * M > NT_CAP) ? NT_CAP : (NJ * M > 64) ? NJ * M : 64;  // threads
  static constexpr int PT1 = (NJ * M + NT - 1) / NT;  // pass-1 tasks per thread
  static constexpr int REALS_TILE = W * RS;
  static constexpr int REALS_Y = NJ * YS * 2;
  static constexpr int REALS_Y3 = THREE ? NJ * YS3 * 2 : 0;
  static constexpr int REALS_Z = NJ * ZS * 2;
  static constexpr int M1 = REALS_TILE > REALS_Y ? REALS_TILE : REALS_Y;
  static constexpr int M2 = M1 > REALS_Y3 ? M1 : REALS_Y3;
  static constexpr int REALS = M2 > REALS_Z ? M2 : REALS_Z;
  static constexpr size_t BYTES = (size_t)REALS * sizeof(T);
};

// cos(2 pi m / 32) from the first octant, exact at the quarter points
__host__ __device__ constexpr double c32oct(int m) {
  return m == 0 ? 1.0
       : m == 1 ? 0.98078528040323043
       : m == 2 ? 0.92387953251128674
       : m == 3 ? 0.83146961230254524
       : m == 4 ? 0.70710678118654752
       : m == 5 ? 0.55557023301960218
       : m == 6 ? 0.38268343236508977
       : m == 7 ? 0.19509032201612826
                : 0.0;
}
__host__ __device__ constexpr double cos32(int m) {
  return (m & 31) <= 8 ? c32oct(m & 31)
       : (m & 31) <= 16 ? -c32oct(16 - (m & 31))
       : (m & 31) <= 24 ? -c32oct((m & 31) - 16)
                        : c32oct(32 - (m & 31));
}
__host__ __device__ constexpr double sin32(int m) { return cos32(8 - m); }

// W_R^m = exp(-+ 2 pi i m / R) for R dividing 32
template <typename T, int R, bool INV>
__host__ __device__ __forceinline__ C2<T> wR(int m) {
  const int q = m * (32 / R);
  return {T(cos32(q)), INV ? T(sin32(q)) : T(-sin32(q))};
}

// R-point DFT in registers, R in {1, 2, 4, 8, 16, 32}; INV selects the exponent sign
// u W_R^m for a literal m: the powers of i as sign changes and swaps (a product with the
// literal 0 of such a twiddle is not folded away under IEEE rules)
template <typename T, int R, bool INV>
__host__ __device__ __forceinline__ C2<T> twR(C2<T> u, int m) {
  const int q = (m * (32 / R)) & 31;
  if (q == 0) return u;
  if (q == 16) return {-u.x, -u.y};
  if (q == 8) return INV ? C2<T>{-u.y, u.x} : C2<T>{u.y, -u.x};   // W = i or -i
  if (q == 24) return INV ? C2<T>{u.y, -u.x} : C2<T>{-u.y, u.x};  // W = -i or i
  return cmul(u, wR<T, R, INV>(m));
}

template <typename T, int R, bool INV>
__host__ __device__ __forceinline__ void dftR(C2<T>* v) {
  if constexpr (R == 2) {
    const C2<T> a = v[0], b = v[1];
    v[0] = {a.x + b.x, a.y + b.y};
    v[1] = {a.x - b.x, a.y - b.y};
  } else if constexpr (R == 4) {
    const C2<T> a0 = {v[0].x + v[2].x, v[0].y + v[2].y};
    const C2<T> a1 = {v[0].x - v[2].x, v[0].y - v[2].y};
    const C2<T> a2 = {v[1].x + v[3].x, v[1].y + v[3].y};
    const C2<T> d = {v[1].x - v[3].x, v[1].y - v[3].y};
    const C2<T> a3 = INV ? C2<T>{-d.y, d.x} : C2<T>{d.y, -d.x};
    v[0] = {a0.x + a2.x, a0.y + a2.y};
    v[1] = {a1.x + a3.x, a1.y + a3.y};
    v[2] = {a0.x - a2.x, a0.y - a2.y};
    v[3] = {a1.x - a3.x, a1.y - a3.y};
  } else if constexpr (R > 4) {
    // R = 4 * B:  n = B n1 + n2, k = k1 + 4 k2
    constexpr int B = R / 4;
    C2<T> t[R];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      C2<T> u[4];
#pragma unroll
      for (int n1 = 0; n1 < 4; ++n1) u[n1] = v[B * n1 + n2];
      dftR<T, 4, INV>(u);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) t[k1 * B + n2] = twR<T, R, INV>(u[k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      C2<T> u[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) u[n2] = t[k1 * B + n2];
      dftR<T, B, INV>(u);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) v[k1 + 4 * k2] = u[k2];
    }
  }
}

__device__ __forceinline__ int perm_src(int n, int N) {  // Makhoul reordering
  return (n < N / 2) ? 2 * n : 2 * (N - 1 - n) + 1;
}
__device__ __forceinline__ int perm_dst(int b, int N) {  // inverse reordering
  return (b & 1) ? N - 1 - (b >> 1) : (b >> 1);
}

// Sources of real pencil samples: pair(j, i) returns sample i of pencils 2j and 2j+1.
template <typename T, int N>
struct LdsSrc {  // tile rows in LDS (row stride N + 1)
  const T* lds;
  __device__ __forceinline__ C2<T> pair(int j, int i) const {
    return {lds[(2 * j) * (N + 1) + i], lds[(2 * j + 1) * (N + 1) + i]};
  }
};
template <typename T>
struct GlobSrc {  // pencils adjacent in memory (x/y passes): one vector load per pair
  const T* g;
  long base, nstride;
  __device__ __forceinline__ C2<T> pair(int j, int i) const {
    return *reinterpret_cast<const C2<T>*>(g + base + (long)i * nstride + 2 * j);
  }
};

// complex FFT input sample n of job j
template <typename T, int N, int KIND, class Src>
__device__ __forceinline__ C2<T> pre_sample(const Src& src, const Tab<T>& tb, int j, int n) {
  if constexpr (KIND == DCT2 || KIND == DST2) {
    const int b = perm_src(n, N);
    C2<T> v = src.pair(j, b);
    if (KIND == DST2 && (b & 1)) v = {-v.x, -v.y};
    return v;
  } else if constexpr (KIND == DCT3 || KIND == DST3) {
    const int k = n;
    // Y_k = X'_k / s_k and Y_{N-k} (Y_N = 0); X' = X (DCT-III) or X reversed (DST-III)
    const int ik = (KIND == DST3) ? N - 1 - k : k;
    const int ir = (KIND == DST3) ? k - 1 : N - k;  // index of X'_{N-k}
    const T s1 = (k == 0) ? tb.is0 : tb.is1;
    const C2<T> y = src.pair(j, ik);
    C2<T> yr = {T(0), T(0)};
    if (k > 0) {
      const T s2 = tb.is1;  // 1 / s_{N-k}, N - k > 0
      const C2<T> t = src.pair(j, ir);
      yr = {t.x * s2, t.y * s2};
    }
    // V = conj(mk_k) * (Y_k - i Y_{N-k}); the two pencils are combined as Va + i Vb
    const C2<T> c = {tb.mk[k].x, -tb.mk[k].y};
    const C2<T> Va = cmul(c, C2<T>{y.x * s1, -yr.x});
    const C2<T> Vb = cmul(c, C2<T>{y.y * s1, -yr.y});
    return {Va.x - Vb.y, Va.y + Vb.x};
  } else {  // DST1: odd extension of length 2N (samples 0 and N are zero)
    if (n == 0 || n == N) return {T(0), T(0)};
    if (n < N) return src.pair(j, n);
    const C2<T> v = src.pair(j, 2 * N - n);
    return {-v.x, -v.y};
  }
}

// Complex FFTs of the W/2 jobs of the tile; on return the spectra are in LDS at
// cb[j * ZS + k] (natural order, length L).  LDS may alias the source (pass-1 samples are
// staged in registers).  Every thread of the block must call it; a block may have more
// threads than Cfg::NT (the extra ones only take part in the barriers).
template <typename T, int N, int KIND, class Sampler>
__device__ void fft_core(T* lds, Sampler&& sample, const Tab<T>& tb);

template <typename T, int N, int KIND, class Src>
__device__ __forceinline__ void fft_tile(T* lds, const Src& src, const Tab<T>& tb) {
  fft_core<T, N, KIND>(lds, [&](int j, int n) { return pre_sample<T, N, KIND>(src, tb, j, n); }, tb);
}

// Pass-1 samples of the thread: z[u][n1] = sample(j, M n1 + m) for its task u = (j, m).
template <typename T, int N, int KIND, class Sampler>
__device__ __forceinline__ void fft_gather(Sampler&& sample,
                                           C2<T> (&z)[TileCfg<T, N, KIND>::PT1][TileCfg<T, N, KIND>::R1]) {
  using S = TileCfg<T, N, KIND>;
  constexpr int NJ = S::NJ, R1 = S::R1, M = S::M, NT = S::NT, TASKS = NJ * M;
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < S::PT1; ++u) {
    const int task = tid + u * NT;
    if ((TASKS % NT == 0 || task < TASKS) && tid < NT) {
      const int j = task % NJ, m = task / NJ;
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) z[u][n1] = sample(j, M * n1 + m);
    }
  }
}

template <typename T, int N, int KIND>
__device__ void fft_core_from(T* lds, C2<T> (&z)[TileCfg<T, N, KIND>::PT1][TileCfg<T, N, KIND>::R1],
                              const Tab<T>& tb);

// Same, with the complex FFT input given directly by sample(j, n) (it may read LDS).
template <typename T, int N, int KIND, class Sampler>
__device__ void fft_core(T* lds, Sampler&& sample, const Tab<T>& tb) {
  using S = TileCfg<T, N, KIND>;
  C2<T> z[S::PT1][S::R1];
  fft_gather<T, N, KIND>(sample, z);
  fft_core_from<T, N, KIND>(lds, z, tb);
}

// Pass 1 of one task (j, n2 = m): R1-point DFT of its samples and the L-point twiddles
template <typename T, int N, int KIND>
__device__ __forceinline__ void fft_pass1_dft(int n2, C2<T> (&z)[TileCfg<T, N, KIND>::R1], const Tab<T>& tb) {
  using S = TileCfg<T, N, KIND>;
  constexpr bool INV = (KIND == DCT3 || KIND == DST3);
  const C2<T>* tw = (S::L == N) ? tb.tw : tb.tw2;
  dftR<T, S::R1, INV>(z);
#pragma unroll
  for (int k1 = 1; k1 < S::R1; ++k1) {
    C2<T> w = tw[n2 * k1];
    if (INV) w.y = -w.y;
    z[k1] = cmul(z[k1], w);
  }
}
// ... and its transposed store
template <typename T, int N, int KIND>
__device__ __forceinline__ void fft_pass1_store(C2<T>* cb, const C2<T> (&z)[TileCfg<T, N, KIND>::R1], int j,
                                                int n2) {
  using S = TileCfg<T, N, KIND>;
#pragma unroll
  for (int k1 = 0; k1 < S::R1; ++k1) cb[j * S::YS + k1 * S::P2 + n2] = z[k1];
}
// Pass 2 of one task (j, k1) of a two-pass FFT: z[k2] = spectrum value k1 + R1 k2 of job j
template <typename T, int N, int KIND>
__device__ __forceinline__ void fft_pass2_dft(const C2<T>* cb, C2<T> (&z)[TileCfg<T, N, KIND>::R2], int j, int k1) {
  using S = TileCfg<T, N, KIND>;
  constexpr bool INV = (KIND == DCT3 || KIND == DST3);
#pragma unroll
  for (int n2 = 0; n2 < S::R2; ++n2) z[n2] = cb[j * S::YS + k1 * S::P2 + n2];
  dftR<T, S::R2, INV>(z);
}
template <typename T, int N, int KIND>
__device__ __forceinline__ void fft_pass2_store(C2<T>* cb, const C2<T> (&z)[TileCfg<T, N, KIND>::R2], int j,
                                                int k1) {
  using S = TileCfg<T, N, KIND>;
#pragma unroll
  for (int k2 = 0; k2 < S::R2; ++k2) cb[j * S::ZS + k1 + S::R1 * k2] = z[k2];
}

// pass 1 of every task: R1-point DFTs over stride-M samples, twiddle, transpose (block barrier
// before the transposed stores, which may overwrite the samples' source, and after them)
template <typename T, int N, int KIND>
__device__ __forceinline__ void fft_pass1_all(C2<T>* cb, C2<T> (&z)[TileCfg<T, N, KIND>::PT1][TileCfg<T, N, KIND>::R1],
                                              const Tab<T>& tb) {
  using S = TileCfg<T, N, KIND>;
  constexpr int NJ = S::NJ, M = S::M, NT = S::NT, TASKS = NJ * M, PT = S::PT1;
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < PT; ++u) {
    const int task = tid + u * NT;
    if ((TASKS % NT == 0 || task < TASKS) && tid < NT) fft_pass1_dft<T, N, KIND>(task / NJ, z[u], tb);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PT; ++u) {
    const int task = tid + u * NT;
    if ((TASKS % NT == 0 || task < TASKS) && tid < NT) fft_pass1_store<T, N, KIND>(cb, z[u], task % NJ, task / NJ);
  }
  __syncthreads();
}

// Three-pass FFTs (R3 > 1): after pass 1, the M-point DFTs of Y[k1][m] (m = R3 m2 + m3) as
// R2-point DFTs over m2 with the M-point twiddles W_M^(m3 k2), a transpose (pass 2), and
// R3-point DFTs over m3 (pass 3); spectrum value k1 + R1 (k2 + R2 k3) in natural order.  Each
// pass ends with a block barrier.
template <typename T, int N, int KIND>
__device__ __forceinline__ void fft3_pass2(C2<T>* cb, const Tab<T>& tb) {
  using S = TileCfg<T, N, KIND>;
  constexpr int NJ = S::NJ, R1 = S::R1, R2 = S::R2, R3 = S::R3, M = S::M, NT = S::NT;
  constexpr bool INV = (KIND == DCT3 || KIND == DST3);
  const C2<T>* tw = (S::L == N) ? tb.tw : tb.tw2;
  const int tid = threadIdx.x;
  constexpr int TASKS = NJ * R1 * R3;
  constexpr int PT = (TASKS + NT - 1) / NT;
  C2<T> zb[PT][R2];
#pragma unroll
  for (int u = 0; u < PT; ++u) {
    const int task = tid + u * NT;
    if ((TASKS % NT == 0 || task < TASKS) && tid < NT) {
      const int j = task % NJ, rest = task / NJ, m3 = rest % R3, k1 = rest / R3;
#pragma unroll
      for (int m2 = 0; m2 < R2; ++m2) zb[u][m2] = cb[j * S::YS + k1 * S::P2 + R3 * m2 + m3];
      dftR<T, R2, INV>(zb[u]);
#pragma unroll
      for (int k2 = 1; k2 < R2; ++k2) {
        C2<T> w = tw[(S::L / M) * m3 * k2];
        if (INV) w.y = -w.y;
        zb[u][k2] = cmul(zb[u][k2], w);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PT; ++u) {
    const int task = tid + u * NT;
    if ((TASKS % NT == 0 || task < TASKS) && tid < NT) {
      const int j = task % NJ, rest = task / NJ, m3 = rest % R3, k1 = rest / R3;
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) cb[j * S::YS3 + (k1 * R2 + k2) * S::P3 + m3] = zb[u][k2];
    }
  }
  __syncthreads();
}
// pass 3 of one task (j, k1, k2): z[k3] = spectrum value k1 + R1 (k2 + R2 k3) of job j
template <typename T, int N, int KIND>
__device__ __forceinline__ void fft3_pass3_task(const C2<T>* cb, C2<T> (&z)[TileCfg<T, N, KIND>::R3], int j, int k1,
                                                int k2) {
  using S = TileCfg<T, N, KIND>;
  constexpr bool INV = (KIND == DCT3 || KIND == DST3);
#pragma unroll
  for (int m3 = 0; m3 < S::R3; ++m3) z[m3] = cb[j * S::YS3 + (k1 * S::R2 + k2) * S::P3 + m3];
  dftR<T, S::R3, INV>(z);
}
template <typename T, int N, int KIND>
__device__ __forceinline__ void fft3_pass3(C2<T>* cb) {
  using S = TileCfg<T, N, KIND>;
  constexpr int NJ = S::NJ, R1 = S::R1, R2 = S::R2, R3 = S::R3, NT = S::NT;
  const int tid = threadIdx.x;
  constexpr int TASKS = NJ * R1 * R2;
  constexpr int PT = (TASKS + NT - 1) / NT;
  C2<T> zc[PT][R3];
#pragma unroll
  for (int u = 0; u < PT; ++u) {
    const int task = tid + u * NT;
    if ((TASKS % NT == 0 || task < TASKS) && tid < NT) {
      const int j = task % NJ, rest = task / NJ, k2 = rest % R2, k1 = rest / R2;
      fft3_pass3_task<T, N, KIND>(cb, zc[u], j, k1, k2);
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PT; ++u) {
    const int task = tid + u * NT;
    if ((TASKS % NT == 0 || task < TASKS) && tid < NT) {
      const int j = task % NJ, rest = task / NJ, k2 = rest % R2, k1 = rest / R2;
#pragma unroll
      for (int k3 = 0; k3 < R3; ++k3) cb[j * S::ZS + k1 + R1 * (k2 + R2 * k3)] = zc[u][k3];
    }
  }
  __syncthreads();
}

// The FFTs from the pass-1 samples already in registers (z is overwritten).
template <typename T, int N, int KIND>
__device__ void fft_core_from(T* lds, C2<T> (&z)[TileCfg<T, N, KIND>::PT1][TileCfg<T, N, KIND>::R1],
                              const Tab<T>& tb) {
  using S = TileCfg<T, N, KIND>;
  constexpr int NJ = S::NJ, R1 = S::R1, R2 = S::R2, R3 = S::R3, NT = S::NT;
  C2<T>* cb = reinterpret_cast<C2<T>*>(lds);
  const int tid = threadIdx.x;
  fft_pass1_all<T, N, KIND>(cb, z, tb);
  if constexpr (R3 > 1) {
    fft3_pass2<T, N, KIND>(cb, tb);
    fft3_pass3<T, N, KIND>(cb);
    return;
  }
  // ---------------- pass 2: R2-point DFTs, natural-order output
  {
    constexpr int TASKS = NJ * R1;
    constexpr int PT = (TASKS + NT - 1) / NT;
    C2<T> z2[PT][R2];
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int task = tid + u * NT;
      if ((TASKS % NT == 0 || task < TASKS) && tid < NT) fft_pass2_dft<T, N, KIND>(cb, z2[u], task % NJ, task / NJ);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int task = tid + u * NT;
      if ((TASKS % NT == 0 || task < TASKS) && tid < NT) fft_pass2_store<T, N, KIND>(cb, z2[u], task % NJ, task / NJ);
    }
    __syncthreads();
  }
}

// Both outputs of index k of job j (pencils 2j and 2j+1) from one read of the spectra.
template <typename T, int N, int KIND>
__device__ __forceinline__ void post_pair(const T* lds, const Tab<T>& tb, int j, int k, T& v0, T& v1) {
  constexpr int ZS = TileCfg<T, N, KIND>::ZS;
  const C2<T>* Z = reinterpret_cast<const C2<T>*>(lds) + j * ZS;
  if constexpr (KIND == DCT2 || KIND == DST2) {
    const int kk = (KIND == DST2) ? N - 1 - k : k;
    const C2<T> a = Z[kk], b = Z[(N - kk) & (N - 1)];
    const C2<T> m = tb.mk[kk];
    const T f = ((kk == 0) ? tb.s0 : tb.s1) * T(0.5);
    // V_a = (a + conj b)/2, V_b = (a - conj b)/(2i); output = sc Re(m V)
    v0 = f * (m.x * (a.x + b.x) - m.y * (a.y - b.y));
    v1 = f * (m.x * (a.y + b.y) - m.y * (b.x - a.x));
  } else if constexpr (KIND == DCT3 || KIND == DST3) {
    const C2<T> z = Z[perm_dst(k, N)];
    const T f = (KIND == DST3 && (k & 1)) ? -(T(1) / T(N)) : (T(1) / T(N));
    v0 = z.x * f;
    v1 = z.y * f;
  } else {
    const C2<T> z = Z[k];
    const T f = (k == 0) ? T(0) : tb.sc[1] * T(0.5);  // sqrt(2/N) / 2
    v0 = -z.y * f;
    v1 = z.x * f;
  }
}

// 16-byte vector of T (global loads and stores of whole vectors)
template <typename T>
struct alignas(16) V16 {
  static constexpr int n = 16 / (int)sizeof(T);
  T a[16 / sizeof(T)];
};

// Output items of a tile after fft_tile.  Axis 2 (pencils contiguous, N apart): item (j, kv)
// covers outputs k = kv*VEC .. kv*VEC+VEC-1 of pencils 2j and 2j+1 (two 16-byte stores, a
// wavefront writes whole pencils).  Axes 0, 1 (pencils adjacent in memory): item (j, k) covers
// output k of pencils 2j and 2j+1 (one 2-element store, a wavefront writes whole 128-byte rows
// of the tile).  Thread t handles items t + u*NT, u < PER.
template <typename T, int N, int KIND>
struct OutItems {
  using S = TileCfg<T, N, KIND>;
  static constexpr int NT = S::NT, NJ = S::NJ, VEC = V16<T>::n;
  static constexpr int NKV = N / VEC;
  static constexpr int COUNT_Z = NJ * NKV, PER_Z = (COUNT_Z + NT - 1) / NT;
  static constexpr int COUNT_XY = NJ * N, PER_XY = (COUNT_XY + NT - 1) / NT;
  __device__ static bool z(int u, int& j, int& k0) {
    const int e = threadIdx.x + u * NT;
    j = e / NKV;
    k0 = (e - j * NKV) * VEC;
    return (COUNT_Z % NT == 0 || e < COUNT_Z) && (int)threadIdx.x < NT;
  }
  __device__ static bool xy(int u, int& j, int& k) {
    const int e = threadIdx.x + u * NT;
    k = e / NJ;
    j = e - k * NJ;
    return (COUNT_XY % NT == 0 || e < COUNT_XY) && (int)threadIdx.x < NT;
  }
  __device__ static void z_values(const T* lds, const Tab<T>& tb, int j, int k0, V16<T>& a, V16<T>& b) {
#pragma unroll
    for (int q = 0; q < VEC; ++q) post_pair<T, N, KIND>(lds, tb, j, k0 + q, a.a[q], b.a[q]);
  }
};

// Tile addressing.  Field layout [x][y][z], z contiguous, N^3 elements.
//  axis 2: tile = W consecutive z-pencils (pencil q = blk*W + p, (x, y) = (q / N, q % N))
//  axis 1: tile = y-pencils at fixed x for W consecutive z  (blk = x * (N/W) + zt)
//  axis 0: tile = x-pencils at fixed y for W consecutive z  (blk = y * (N/W) + zt)
struct TileAddr {
  long base, pstride, nstride;
};

template <int W, int N>
__device__ __forceinline__ TileAddr tile_addr(int axis, int blk) {
  TileAddr a;
  if (axis == 2) {
    a.base = (long)blk * W * N;
    a.pstride = N;
    a.nstride = 1;
  } else {
    const int outer = blk / (N / W), zt = blk % (N / W);
    if (axis == 1) {
      a.base = (long)outer * N * N + zt * W;
      a.nstride = N;
    } else {
      a.base = (long)outer * N + zt * W;
      a.nstride = (long)N * N;
    }
    a.pstride = 1;
  }
  return a;
}

// element e of the tile in coalescing order -> (p, n)
template <int W, int N>
__device__ __forceinline__ void tile_elem(int axis, int e, int& p, int& n) {
  if (axis == 2) {
    p = e / N;
    n = e - p * N;
  } else {
    n = e / W;
    p = e - n * W;
  }
}

}  // namespace kfbi
