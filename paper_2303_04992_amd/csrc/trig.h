// Pencil sine/cosine transforms in LDS for gfx950.
//
// The FFT-based Poisson solver of the paper (Sec. 4.2, items ii-iii) needs, per axis, the
// orthonormal DCT-II / DST-II (length N, cell-centred and tangential face axes), their
// inverses DCT-III / DST-III, and the DST-I (length N-1, the face-normal axis).  Here every
// transform of two real pencils is one complex FFT: for the DCT/DST pair the real pencils
// are reordered (even samples ascending, odd samples descending) so that a length-N complex
// FFT plus one twiddle per output gives the cosine sums (Makhoul's algorithm); DST-II is the
// DCT-II of the sign-alternated pencil read backwards; DST-I is the FFT of the odd extension
// of length 2N.  The complex FFT is a Stockham autosort FFT with radix-4 stages (and one
// radix-2 stage when log2 L is odd), register staged so that one LDS buffer holds the data.
//
// A workgroup owns a tile of W real pencils (W*sizeof(T) = 128 bytes, so every row of the
// tile along the contiguous z axis is one 128-byte segment), stored in LDS as rows of length
// N + 1 (the padding breaks bank conflicts of the strided x/y loads).
#pragma once
#include <hip/hip_runtime.h>

namespace kfbi {

constexpr int NT = 256;  // threads per workgroup of every transform kernel

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
};

template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// tile width: one 128-byte row segment, at most the grid size
template <typename T, int N>
struct TileShape {
  static constexpr int W = (int)(128 / sizeof(T)) < N ? (int)(128 / sizeof(T)) : N;
};

template <typename T, int N, int KIND>
struct TileLDS {
  static constexpr int W = TileShape<T, N>::W;
  static constexpr int RS = N + 1;
  static constexpr int L = (KIND == DST1) ? 2 * N : N;
  static constexpr int NJ = W / 2;
  static constexpr int REALS_TILE = W * RS;
  static constexpr int REALS_CPLX = NJ * L * 2;
  static constexpr int REALS = REALS_TILE > REALS_CPLX ? REALS_TILE : REALS_CPLX;
  static constexpr size_t BYTES = (size_t)REALS * sizeof(T);
};

// radix-R DFT in registers (R = 2 or 4); INV selects the sign of the exponent
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(C2<T>* v) {
  if constexpr (R == 2) {
    C2<T> a = v[0], b = v[1];
    v[0] = {a.x + b.x, a.y + b.y};
    v[1] = {a.x - b.x, a.y - b.y};
  } else {
    C2<T> a0 = {v[0].x + v[2].x, v[0].y + v[2].y};
    C2<T> a1 = {v[0].x - v[2].x, v[0].y - v[2].y};
    C2<T> a2 = {v[1].x + v[3].x, v[1].y + v[3].y};
    C2<T> d = {v[1].x - v[3].x, v[1].y - v[3].y};
    C2<T> a3 = INV ? C2<T>{-d.y, d.x} : C2<T>{d.y, -d.x};
    v[0] = {a0.x + a2.x, a0.y + a2.y};
    v[1] = {a1.x + a3.x, a1.y + a3.y};
    v[2] = {a0.x - a2.x, a0.y - a2.y};
    v[3] = {a1.x - a3.x, a1.y - a3.y};
  }
}

// one Stockham stage over NJ complex pencils of length L held in LDS
template <typename T, int L, int NJ, int R, int NS, bool INV>
__device__ __forceinline__ void stockham_stage(C2<T>* cb, const C2<T>* tw) {
  constexpr int NBP = L / R;  // butterflies per pencil
  constexpr int NB = NJ * NBP;
  constexpr int PB = (NB + NT - 1) / NT;
  const int tid = threadIdx.x;
  C2<T> v[PB][R];
#pragma unroll
  for (int u = 0; u < PB; ++u) {
    const int b = tid + u * NT;
    if (NB % NT == 0 || b < NB) {
      const int job = b / NBP, j = b - job * NBP, jm = j % NS;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        C2<T> a = cb[job * L + j + t * NBP];
        if (NS > 1) {
          C2<T> w = tw[(L / (NS * R)) * jm * t];
          if (INV) w.y = -w.y;
          a = cmul(a, w);
        }
        v[u][t] = a;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PB; ++u) {
    const int b = tid + u * NT;
    if (NB % NT == 0 || b < NB) {
      const int job = b / NBP, j = b - job * NBP, jm = j % NS;
      dft<T, R, INV>(v[u]);
      const int idxD = (j / NS) * NS * R + jm;
#pragma unroll
      for (int t = 0; t < R; ++t) cb[job * L + idxD + t * NS] = v[u][t];
    }
  }
  __syncthreads();
}

template <typename T, int L, int NJ, int NS, bool INV>
__device__ __forceinline__ void fft_stages(C2<T>* cb, const C2<T>* tw) {
  if constexpr (NS < L) {
    constexpr int R = (NS * 4 <= L) ? 4 : 2;
    stockham_stage<T, L, NJ, R, NS, INV>(cb, tw);
    fft_stages<T, L, NJ, NS * R, INV>(cb, tw);
  }
}

__device__ __forceinline__ int perm_src(int n, int N) {  // Makhoul reordering
  return (n < N / 2) ? 2 * n : 2 * (N - 1 - n) + 1;
}
__device__ __forceinline__ int perm_dst(int b, int N) {  // inverse reordering
  return (b & 1) ? N - 1 - (b >> 1) : (b >> 1);
}

// Transform the W real pencils of the tile in place (tile row p at lds[p * RS]).
template <typename T, int N, int KIND>
__device__ void transform_tile(T* lds, const Tab<T>& tb) {
  using S = TileLDS<T, N, KIND>;
  constexpr int W = S::W, RS = S::RS, L = S::L, NJ = S::NJ;
  constexpr bool INV = (KIND == DCT3 || KIND == DST3);
  C2<T>* cb = reinterpret_cast<C2<T>*>(lds);
  const int tid = threadIdx.x;
  // ---------------- pre-processing: real tile -> complex sequences
  {
    constexpr int CNT = NJ * L;
    constexpr int PER = (CNT + NT - 1) / NT;
    C2<T> r[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NT;
      if (CNT % NT == 0 || e < CNT) {
        const int j = e / L, n = e - j * L;
        const T* ra = lds + (2 * j) * RS;
        const T* rb = lds + (2 * j + 1) * RS;
        C2<T> z;
        if constexpr (KIND == DCT2 || KIND == DST2) {
          const int b = perm_src(n, N);
          T va = ra[b], vb = rb[b];
          if (KIND == DST2 && (b & 1)) {
            va = -va;
            vb = -vb;
          }
          z = {va, vb};
        } else if constexpr (KIND == DCT3 || KIND == DST3) {
          const int k = n;
          // Y_k = X'_k / s_k and Y_{N-k} (Y_N = 0); X' = X (DCT-III) or X reversed (DST-III)
          const int ik = (KIND == DST3) ? N - 1 - k : k;
          const int ir = (KIND == DST3) ? k - 1 : N - k;  // index of X'_{N-k}
          const T s1 = tb.isc[k];
          const T s2 = (k > 0) ? tb.isc[N - k] : T(0);
          const T ya = ra[ik] * s1, yb = rb[ik] * s1;
          const T yra = (k > 0) ? ra[ir] * s2 : T(0);
          const T yrb = (k > 0) ? rb[ir] * s2 : T(0);
          // V = conj(mk_k) * (Y_k - i Y_{N-k})
          const C2<T> c = {tb.mk[k].x, -tb.mk[k].y};
          const C2<T> Va = cmul(c, C2<T>{ya, -yra});
          const C2<T> Vb = cmul(c, C2<T>{yb, -yrb});
          z = {Va.x - Vb.y, Va.y + Vb.x};
        } else {  // DST1: odd extension of length 2N (samples 0 and N are zero)
          T va, vb;
          if (n == 0 || n == N) {
            va = vb = T(0);
          } else if (n < N) {
            va = ra[n];
            vb = rb[n];
          } else {
            va = -ra[2 * N - n];
            vb = -rb[2 * N - n];
          }
          z = {va, vb};
        }
        r[u] = z;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NT;
      if (CNT % NT == 0 || e < CNT) cb[e] = r[u];
    }
    __syncthreads();
  }
  // ---------------- complex FFT of length L
  fft_stages<T, L, NJ, 1, INV>(cb, (L == N) ? tb.tw : tb.tw2);
  // ---------------- post-processing: complex spectra -> real tile
  {
    constexpr int CNT = W * N;
    constexpr int PER = (CNT + NT - 1) / NT;
    T o[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NT;
      if (CNT % NT == 0 || e < CNT) {
        const int p = e / N, k = e - p * N;
        const int j = p >> 1, which = p & 1;
        const C2<T>* Z = cb + j * L;
        T val;
        if constexpr (KIND == DCT2 || KIND == DST2) {
          const int kk = (KIND == DST2) ? N - 1 - k : k;
          const C2<T> a = Z[kk], b = Z[(N - kk) & (N - 1)];
          C2<T> V;
          if (which == 0)
            V = {(a.x + b.x) * T(0.5), (a.y - b.y) * T(0.5)};
          else
            V = {(a.y + b.y) * T(0.5), (b.x - a.x) * T(0.5)};
          const C2<T> m = tb.mk[kk];
          val = tb.sc[kk] * (m.x * V.x - m.y * V.y);
        } else if constexpr (KIND == DCT3 || KIND == DST3) {
          const C2<T> z = Z[perm_dst(k, N)];
          val = (which ? z.y : z.x) * (T(1) / T(N));
          if (KIND == DST3 && (k & 1)) val = -val;
        } else {
          const C2<T> z = Z[k];
          const T y = which ? z.x * T(0.5) : -z.y * T(0.5);
          val = (k == 0) ? T(0) : y * tb.sc[1];  // sqrt(2/N)
        }
        o[u] = val;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * NT;
      if (CNT % NT == 0 || e < CNT) {
        const int p = e / N, k = e - p * N;
        lds[p * RS + k] = o[u];
      }
    }
    __syncthreads();
  }
}

// Tile addressing.  Field layout [x][y][z], z contiguous, N^3 elements.
//  axis 2: tile = W consecutive z-pencils (pencil q = blk*W + p, (x, y) = (q / N, q % N))
//  axis 1: tile = y-pencils at fixed x for W consecutive z  (blk = x * (N/W) + zt)
//  axis 0: tile = x-pencils at fixed y for W consecutive z  (blk = y * (N/W) + zt)
struct TileAddr {
  long base, pstride, nstride;
};

template <typename T, int N>
__device__ __forceinline__ TileAddr tile_addr(int axis, int blk) {
  constexpr int W = TileShape<T, N>::W;
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
template <typename T, int N>
__device__ __forceinline__ void tile_elem(int axis, int e, int& p, int& n) {
  constexpr int W = TileShape<T, N>::W;
  if (axis == 2) {
    p = e / N;
    n = e - p * N;
  } else {
    n = e / W;
    p = e - n * W;
  }
}

}  // namespace kfbi
