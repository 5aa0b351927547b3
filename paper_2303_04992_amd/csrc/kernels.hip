// Device kernels of the KFBI operator evaluation on gfx950.
//
// MAC solve (Sec. 4.2 items i-iii of the paper).  With A_u = -mu Delta_h on the face grid
// T^m diagonalised by T_m = (DST-I along m) x (DST-II along the two other axes), and the
// MAC gradient satisfying T_m G_m = -sigma_m C_m with C_m = (DCT-II along m) x (DST-II
// elsewhere) and sigma_k = (2/h) sin(pi k / 2N), the Schur complement is
//     S = G^T A_u^{-1} G + c I = sum_m C_m^T [sigma_{k_m}^2 / Lambda_m] C_m + c I,
// so every CG iteration is three mixed sine/cosine transforms of the pressure, a diagonal
// scaling and three inverse transforms (no separate gradient/divergence stencil passes).
// The right-hand side is P(F_p - sum_m C_m^T [sigma/Lambda_m] T_m F_m) and the velocity
// back-substitution u_m = T_m^T [(T_m F_m + sigma C_m p) / Lambda_m].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

#include "kernels.h"
#include "trig.h"

namespace kfbi {

// ---------------------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------------------
template <typename T>
static Tab<T> tab_of(const DevTables<T>& d) {
  Tab<T> t;
  t.tw = reinterpret_cast<const C2<T>*>(d.tw);
  t.tw2 = reinterpret_cast<const C2<T>*>(d.tw2);
  t.mk = reinterpret_cast<const C2<T>*>(d.mk);
  t.sc = d.sc;
  t.isc = d.isc;
  t.s0 = d.s0;
  t.s1 = d.s1;
  t.is0 = d.is0;
  t.is1 = d.is1;
  t.sg2 = d.sg2;
  t.sg2s = d.sg2s;
  return t;
}

// Batched launches (see Bat): the right-hand side of a block is blockIdx.z; its work buffers lie
// blockIdx.z * A bytes after those of right-hand side 0, its caller arrays blockIdx.z * U
// elements further; null pointers stay null.
__device__ __forceinline__ bool rhs_skipped(const Bat& b) { return b.act != nullptr && b.act[blockIdx.z] == 0; }
template <typename P>
__device__ __forceinline__ P wb(P p, const Bat& b) {
  return p ? reinterpret_cast<P>(reinterpret_cast<uintptr_t>(p) + (uint64_t)blockIdx.z * (uint64_t)b.A) : p;
}
template <typename P>
__device__ __forceinline__ P ub(P p, const Bat& b) {
  return p ? p + (int64_t)blockIdx.z * b.U : p;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// deterministic block sum of NT threads (4 wavefronts); result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[w];
  return r;
}

// four block sums with one exchange through LDS (sh holds 4 * waves doubles); the totals are
// valid in thread 0
__device__ __forceinline__ void block_sum4(double (&v)[4], double* sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 4; ++c) v[c] = wave_sum(v[c]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) sh[4 * wid + c] = v[c];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double r = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += sh[4 * w + c];
      v[c] = r;
    }
}

constexpr int EW_NT = 256;  // threads per block of the elementwise and reduction kernels

// Upper bound of the threads of a transform block at grid size N (TileCfg::NT): 512 from
// N = 512 on, where a 256-thread block would hold 32 complex values per thread.
template <int N>
constexpr int tile_nt_max() {
  return N >= 512 ? 512 : 256;
}

// Minimum waves per SIMD a transform kernel is compiled for (amdgpu_waves_per_eu; 1 = the
// compiler's choice).  Float32 tiles from N = 128 on are held to four (at most 128 registers): at
// 512 a block has 512 threads, so one register above 128 leaves a single block per compute unit
// where the LDS holds two (z inverse 129, DST-I pass 134 registers as compiled otherwise).  The
// fused x passes of the right-hand side and back-substitution (136-154 registers) then spill a
// few registers, which pays only at 512.
template <typename T, int N>
constexpr int tile_waves() {
  return (sizeof(T) == 4 && N >= 128) ? 4 : 1;
}
template <typename T, int N>
constexpr int xfuse_waves() {
  return (sizeof(T) == 4 && N >= 512) ? 4 : 1;
}

// Contiguous z tile (W pencils of N, 16-byte aligned) -> LDS rows of stride N + 1.  Every
// load of the thread is issued before the first LDS write (vector loads, unrolled).
template <typename T, int N, int NT>
__device__ __forceinline__ void load_tile_z(T* lds, const T* __restrict__ g) {
  constexpr int W = TileCfg<T, N, DCT2>::W, RS = N + 1, VEC = V16<T>::n;
  constexpr int NV = W * N / VEC, PER = (NV + NT - 1) / NT;
  V16<T> v[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * NT;
    if (NV % NT == 0 || e < NV) v[u] = reinterpret_cast<const V16<T>*>(g)[e];
  }
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * NT;
    if (NV % NT == 0 || e < NV) {
      const int p = (e * VEC) / N, n = (e * VEC) - p * N;
#pragma unroll
      for (int q = 0; q < VEC; ++q) lds[p * RS + n + q] = v[u].a[q];
    }
  }
  __syncthreads();
}


// ---------------------------------------------------------------------------------------
// Persistent, software-pipelined transform passes.  A block owns tiles blockIdx.x,
// blockIdx.x + gridDim.x, ...; the raw rows of its next tile are requested into registers
// right after the current tile has been staged in LDS, so they arrive while the current tile
// is transformed.  The transform tables are copied to LDS once per block, so that the
// transform phase waits on LDS only (a table read from global memory would also wait for the
// outstanding prefetch, the vector-memory counter being in order).
// ---------------------------------------------------------------------------------------
template <typename T, int N, int KIND>
struct PipeCfg {
  using S = TileCfg<T, N, KIND>;
  static constexpr size_t TAB_OFF = (S::BYTES + 15) / 16 * 16;
  static constexpr size_t BYTES = TAB_OFF + (size_t)(S::L + N) * sizeof(C2<T>);
  static constexpr int NPAIR = S::NJ * N;                  // element pairs of a tile
  static constexpr int PER = (NPAIR + S::NT - 1) / S::NT;  // per thread
};

// twiddles (tw or tw2) and mk in LDS (the orthonormal scales travel as the scalars of Tab)
template <typename T, int N, int KIND>
__device__ __forceinline__ Tab<T> tables_to_lds(unsigned char* smem, const Tab<T>& g) {
  using S = TileCfg<T, N, KIND>;
  C2<T>* ltw = reinterpret_cast<C2<T>*>(smem + PipeCfg<T, N, KIND>::TAB_OFF);
  C2<T>* lmk = ltw + S::L;
  const C2<T>* gtw = (S::L == N) ? g.tw : g.tw2;
  for (int i = threadIdx.x; i < S::L; i += blockDim.x) ltw[i] = gtw[i];
  for (int i = threadIdx.x; i < N; i += blockDim.x) lmk[i] = g.mk[i];
  Tab<T> t = g;
  t.tw = ltw;
  t.tw2 = ltw;
  t.mk = lmk;
  return t;
}

// The same tables (layout of PipeCfg) for one-tile kernels, in two steps: request() reads
// the entries into registers before the kernel requests its samples, publish() writes them to
// LDS once they (and not the samples, requested later) have arrived.  Used only where the
// extra LDS keeps the resident blocks per compute unit (of the sizes here, float32 at N = 256).
template <typename T, int N, int KIND>
struct TabStage {
  using S = TileCfg<T, N, KIND>;
  using P = PipeCfg<T, N, KIND>;
  static constexpr bool ON = sizeof(T) == 4 && P::BYTES <= 163840 && 163840 / P::BYTES >= 163840 / S::BYTES;
  static constexpr size_t BYTES = ON ? P::BYTES : S::BYTES;
  static constexpr int NT = S::NT, PL = (S::L + NT - 1) / NT, PN = (N + NT - 1) / NT;
  C2<T> rtw[ON ? PL : 1], rmk[ON ? PN : 1];
  __device__ __forceinline__ void request(const Tab<T>& g) {
    if constexpr (ON) {
      const C2<T>* gtw = (S::L == N) ? g.tw : g.tw2;
#pragma unroll
      for (int u = 0; u < PL; ++u) {
        const int i = threadIdx.x + u * NT;
        if (i < S::L) rtw[u] = gtw[i];
      }
#pragma unroll
      for (int u = 0; u < PN; ++u) {
        const int i = threadIdx.x + u * NT;
        if (i < N) rmk[u] = g.mk[i];
      }
    }
  }
  // writes the entries to LDS (the caller synchronises the block before they are read) and
  // returns the tables to read: the LDS copies, or g itself when the stage is off
  __device__ __forceinline__ Tab<T> publish(unsigned char* smem, const Tab<T>& g) const {
    if constexpr (ON) {
      C2<T>* ltw = reinterpret_cast<C2<T>*>(smem + P::TAB_OFF);
      C2<T>* lmk = ltw + S::L;
#pragma unroll
      for (int u = 0; u < PL; ++u) {
        const int i = threadIdx.x + u * NT;
        if (i < S::L) ltw[i] = rtw[u];
      }
#pragma unroll
      for (int u = 0; u < PN; ++u) {
        const int i = threadIdx.x + u * NT;
        if (i < N) lmk[i] = rmk[u];
      }
    }
    return view(smem, g);
  }
  __device__ __forceinline__ static Tab<T> view(unsigned char* smem, const Tab<T>& g) {
    if constexpr (ON) {
      C2<T>* ltw = reinterpret_cast<C2<T>*>(smem + P::TAB_OFF);
      Tab<T> t = g;
      t.tw = ltw;
      t.tw2 = ltw;
      t.mk = ltw + S::L;
      return t;
    } else {
      return g;
    }
  }
};

// raw element pairs (pencils 2j, 2j+1 at sample n) of an x or y tile: pair e -> (n, j) = (e / NJ, e % NJ)
template <typename T, int N, int KIND>
__device__ __forceinline__ void fetch_xy(const T* g, const TileAddr& a, C2<T> (&raw)[PipeCfg<T, N, KIND>::PER]) {
  using S = TileCfg<T, N, KIND>;
  using P = PipeCfg<T, N, KIND>;
#pragma unroll
  for (int u = 0; u < P::PER; ++u) {
    const int e = threadIdx.x + u * S::NT;
    if ((P::NPAIR % S::NT == 0 || e < P::NPAIR) && (int)threadIdx.x < S::NT) {
      const int n = e / S::NJ, j = e - n * S::NJ;
      raw[u] = *reinterpret_cast<const C2<T>*>(g + a.base + (long)n * a.nstride + 2 * j);
    }
  }
}
template <typename T, int N, int KIND>
__device__ __forceinline__ void stage_xy(T* lds, const C2<T> (&raw)[PipeCfg<T, N, KIND>::PER]) {
  using S = TileCfg<T, N, KIND>;
  using P = PipeCfg<T, N, KIND>;
#pragma unroll
  for (int u = 0; u < P::PER; ++u) {
    const int e = threadIdx.x + u * S::NT;
    if ((P::NPAIR % S::NT == 0 || e < P::NPAIR) && (int)threadIdx.x < S::NT) {
      const int n = e / S::NJ, j = e - n * S::NJ;
      lds[(2 * j) * (N + 1) + n] = raw[u].x;
      lds[(2 * j + 1) * (N + 1) + n] = raw[u].y;
    }
  }
}

template <typename T, int N, int KIND>
__global__ __launch_bounds__(tile_nt_max<N>()) void k_pass_pipe(const T* in, T* out, int axis, int ntiles, Tab<T> tg, Bat bt) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (rhs_skipped(bt)) return;
  in = wb(in, bt);
  out = wb(out, bt);
  T* lds = reinterpret_cast<T*>(smem);
  using S = TileCfg<T, N, KIND>;
  constexpr int W = S::W;
  const Tab<T> tb = tables_to_lds<T, N, KIND>(smem, tg);
  C2<T> raw[PipeCfg<T, N, KIND>::PER];
  int tile = blockIdx.x;
  if (tile < ntiles) fetch_xy<T, N, KIND>(in, tile_addr<W, N>(axis, tile), raw);
  for (; tile < ntiles; tile += gridDim.x) {
    __syncthreads();  // the previous tile's outputs have been read from LDS
    stage_xy<T, N, KIND>(lds, raw);
    __syncthreads();
    if (tile + (int)gridDim.x < ntiles) fetch_xy<T, N, KIND>(in, tile_addr<W, N>(axis, tile + gridDim.x), raw);
    fft_tile<T, N, KIND>(lds, LdsSrc<T, N>{lds}, tb);
    const TileAddr a = tile_addr<W, N>(axis, tile);
    store_xy_outputs<T, N, KIND>(lds, tb, out + a.base, a.nstride);
  }
}

// resident blocks of a persistent launch: compute units x blocks per unit (occupancy query)
static int cu_count() {
  static std::atomic<int> n[64];  // per device; 0 = not queried yet (racing threads store the same value)
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int v = n[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
    n[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}
// (per_cu caches the occupancy query of one kernel; the caller keeps it in a static, and
// racing threads store the same value)
template <typename K>
static int persistent_blocks(K kernel, int threads, size_t lds_bytes, int ntiles, std::atomic<int>& per_cu) {
  int v = per_cu.load(std::memory_order_relaxed);
  if (v < 1) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kernel, threads, lds_bytes) != hipSuccess || v < 1) v = 1;
    per_cu.store(v, std::memory_order_relaxed);
  }
  return std::max(1, std::min(ntiles, cu_count() * v));
}

// ---------------------------------------------------------------------------------------
// generic transform pass: out (+)= transform_KIND(in) along axis
// ---------------------------------------------------------------------------------------
// (in may equal out: a block reads its whole tile before it writes any output)
// pmask (may be null; axes 1 and 2 only): the input is zero outside the z-pencils (x, y) whose
// byte pmask[x N + y] has bit mbit set (xmask[x]: the same bits or-ed over y).  A tile without
// such a pencil (axis 2), or of a plane x without one (axis 1: after the z transform a flagged
// pencil fills its whole plane), has a zero transform: it is written as zeros (or, accumulating,
// left as it is) without being read.
template <typename T, int N, int KIND, bool ACC>
__global__ __launch_bounds__(tile_nt_max<N>()) __attribute__((amdgpu_waves_per_eu(tile_waves<T, N>()))) void k_pass(const T* in, T* out, int axis, Tab<T> tb, Bat bt,
                                                const uint8_t* __restrict__ pmask, const uint8_t* __restrict__ xmask,
                                                int mbit) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (rhs_skipped(bt)) return;
  in = wb(in, bt);
  out = wb(out, bt);
  T* lds = reinterpret_cast<T*>(smem);
  using S = TileCfg<T, N, KIND>;
  using O = OutItems<T, N, KIND>;
  constexpr int W = S::W, NT = S::NT;
  const TileAddr a = tile_addr<W, N>(axis, blockIdx.x);
  if (pmask && axis != 0) {
    unsigned any = 0;
    if (axis == 2) {
#pragma unroll
      for (int p = 0; p < W; ++p) any |= pmask[(int64_t)blockIdx.x * W + p];
    } else {
      any = xmask[blockIdx.x / (N / W)];
    }
    if (!((any >> mbit) & 1u)) {
      if constexpr (!ACC) {
        if (axis == 2) {
          constexpr int NV = W * N / V16<T>::n;
          V16<T> zero;
#pragma unroll
          for (int q = 0; q < V16<T>::n; ++q) zero.a[q] = T(0);
          for (int e = threadIdx.x; e < NV; e += blockDim.x) reinterpret_cast<V16<T>*>(out + a.base)[e] = zero;
        } else {
          C2<T>* o = reinterpret_cast<C2<T>*>(out + a.base);
          const long ns = a.nstride / 2;
          for (int e = threadIdx.x; e < N * S::NJ; e += blockDim.x) o[(e / S::NJ) * ns + e % S::NJ] = C2<T>{T(0), T(0)};
        }
      }
      return;
    }
  }
  // forward kinds: the tables are requested before the samples and read from LDS (TabStage)
  using TS = TabStage<T, N, KIND>;
  constexpr bool STAGE = (KIND == DCT2 || KIND == DST2 || KIND == DST1) && TS::ON;
  TS ts;
  if constexpr (STAGE) ts.request(tb);
  Tab<T> tl = tb;
  if (axis == 2) {
    if constexpr (STAGE) {
      constexpr int VEC = V16<T>::n, NV = W * N / VEC, PV = (NV + NT - 1) / NT;
      V16<T> v[PV];
#pragma unroll
      for (int u = 0; u < PV; ++u) {
        const int e = threadIdx.x + u * NT;
        if (NV % NT == 0 || e < NV) v[u] = reinterpret_cast<const V16<T>*>(in + a.base)[e];
      }
      tl = ts.publish(smem, tb);
#pragma unroll
      for (int u = 0; u < PV; ++u) {
        const int e = threadIdx.x + u * NT;
        if (NV % NT == 0 || e < NV) {
          const int p = (e * VEC) / N, n = (e * VEC) - p * N;
#pragma unroll
          for (int q = 0; q < VEC; ++q) lds[p * (N + 1) + n + q] = v[u].a[q];
        }
      }
      __syncthreads();
    } else {
      load_tile_z<T, N, NT>(lds, in + a.base);
    }
    fft_tile<T, N, KIND>(lds, LdsSrc<T, N>{lds}, tl);
    V16<T>* o = reinterpret_cast<V16<T>*>(out + a.base);
    constexpr int RV = N / O::VEC;  // vectors per pencil
    V16<T> old[ACC ? 2 * O::PER_Z : 1];
    if constexpr (ACC) {
#pragma unroll
      for (int u = 0; u < O::PER_Z; ++u) {
        int j, k0;
        if (O::z(u, j, k0)) {
          old[2 * u] = o[(2 * j) * RV + k0 / O::VEC];
          old[2 * u + 1] = o[(2 * j + 1) * RV + k0 / O::VEC];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < O::PER_Z; ++u) {
      int j, k0;
      if (O::z(u, j, k0)) {
        V16<T> v0, v1;
        O::z_values(lds, tl, j, k0, v0, v1);
        if constexpr (ACC) {
#pragma unroll
          for (int q = 0; q < O::VEC; ++q) {
            v0.a[q] += old[2 * u].a[q];
            v1.a[q] += old[2 * u + 1].a[q];
          }
        }
        o[(2 * j) * RV + k0 / O::VEC] = v0;
        o[(2 * j + 1) * RV + k0 / O::VEC] = v1;
      }
    }
  } else {
    const GlobSrc<T> src{in, a.base, a.nstride};
    if constexpr (STAGE) {
      C2<T> z[S::PT1][S::R1];
      fft_gather<T, N, KIND>([&](int j, int n) { return pre_sample<T, N, KIND>(src, tb, j, n); }, z);
      tl = ts.publish(smem, tb);
      __syncthreads();
      fft_core_from<T, N, KIND>(lds, z, tl);
    } else {
      fft_tile<T, N, KIND>(lds, src, tb);
    }
    C2<T>* o = reinterpret_cast<C2<T>*>(out + a.base);
    const long ns = a.nstride / 2;  // in units of element pairs
    C2<T> old[ACC ? O::PER_XY : 1];
    if constexpr (ACC) {
#pragma unroll
      for (int u = 0; u < O::PER_XY; ++u) {
        int j, k;
        if (O::xy(u, j, k)) old[u] = o[k * ns + j];
      }
    }
#pragma unroll
    for (int u = 0; u < O::PER_XY; ++u) {
      int j, k;
      if (O::xy(u, j, k)) {
        C2<T> v;
        post_pair<T, N, KIND>(lds, tl, j, k, v.x, v.y);
        if constexpr (ACC) {
          v.x += old[u].x;
          v.y += old[u].y;
        }
        o[k * ns + j] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// fused Schur x-pass of component mc: forward x (KF), spectral weight sigma^2/Lambda,
// inverse x (KI), in place.  Between the two FFTs the forward post-processing, the weight
// and the inverse pre-processing are applied together on each spectral pair (k, N-k) of a
// job in registers: with V_q = (Z_q + conj Z_{N-q})/2 (pencil a) or
// (Z_q - conj Z_{N-q})/(2i) (pencil b), the inverse input is built from
// Y_q = omega_q Re(e^{-i pi q/2N} V_q), omega_q = w(q) (cosine) or w(N-1-q) (sine), the
// orthonormal scale factors cancelling; V'_q = e^{+i pi q/2N}(Y_q - i Y_{N-q}), Y_N = 0,
// Z'_q = V'^a_q + i V'^b_q.
// ---------------------------------------------------------------------------------------
// one tile: forward x from the pass-1 samples already in registers, weight, inverse x, store
template <typename T, int N, int KF, int KI>
__device__ void xmid_tile(T* lds, T* field, int tile, int mc, double mu, const Tab<T>& tb,
                          C2<T> (&zs)[TileCfg<T, N, KF>::PT1][TileCfg<T, N, KF>::R1]) {
  using S = TileCfg<T, N, KF>;
  constexpr int W = S::W, NJ = S::NJ, ZS = S::ZS, NT = S::NT;
  const TileAddr a = tile_addr<W, N>(0, tile);
  const int yi = tile / (N / W), z0 = (tile % (N / W)) * W;
  fft_core_from<T, N, KF>(lds, zs, tb);
  C2<T>* cb = reinterpret_cast<C2<T>*>(lds);
  constexpr int PAIRS = N / 2 + 1;
  static_assert(NT % NJ == 0, "the job of a thread is fixed across the loop");
  // y and z eigenvalues of the thread's two pencils (its job j = threadIdx.x % NJ is fixed)
  const int jt = threadIdx.x % NJ;
  const T ly = (mc == 1) ? tb.sg2[yi] : tb.sg2s[yi];
  T lz[2];
#pragma unroll
  for (int w = 0; w < 2; ++w) lz[w] = (mc == 2) ? tb.sg2[z0 + 2 * jt + w] : tb.sg2s[z0 + 2 * jt + w];
  // the factor 1/2 of V below is folded into the weight denominators
  const T mu2 = T(2 * mu);
  constexpr int PER = (NJ * PAIRS + NT - 1) / NT;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int t = threadIdx.x + u * NT;
    if (t >= NJ * PAIRS) break;
    const int j = jt, k = t / NJ;
    const int kr = (N - k) & (N - 1);
    const C2<T> Zk = cb[j * ZS + k], Zr = cb[j * ZS + kr];
    // weights sigma_mc^2 / Lambda_mc of the two pencils at DCT-domain indices k and kr;
    // x is the cosine axis for mc = 0 and a sine axis otherwise
    T om[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int q = h ? kr : k;
      const int mode = (KF == DST2) ? N - 1 - q : q;
      const T lx = (mc == 0) ? tb.sg2[mode] : tb.sg2s[mode];
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const T num = (mc == 0) ? lx : (mc == 1) ? ly : lz[w];
        const T den = mu2 * (lx + ly + lz[w]);
        if constexpr (sizeof(T) == 4)
          om[w][h] = num * __builtin_amdgcn_rcpf(den);  // 1 ulp: the float32 inner solve
        else
          om[w][h] = num / den;
      }
    }
    const C2<T> mkk = tb.mk[k], mkr = tb.mk[kr];
    const C2<T> Vak = {Zk.x + Zr.x, Zk.y - Zr.y};  // 2 V^a_k
    const C2<T> Vbk = {Zk.y + Zr.y, Zr.x - Zk.x};  // 2 V^b_k
    const C2<T> Var = {Zr.x + Zk.x, Zr.y - Zk.y};
    const C2<T> Vbr = {Zr.y + Zk.y, Zk.x - Zr.x};
    const T Yak = om[0][0] * (mkk.x * Vak.x - mkk.y * Vak.y);
    const T Ybk = om[1][0] * (mkk.x * Vbk.x - mkk.y * Vbk.y);
    const T Yar = (k == 0) ? T(0) : om[0][1] * (mkr.x * Var.x - mkr.y * Var.y);
    const T Ybr = (k == 0) ? T(0) : om[1][1] * (mkr.x * Vbr.x - mkr.y * Vbr.y);
    // V'_k = conj(mk_k)(Y_k - i Y_{N-k}),  V'_{N-k} = conj(mk_{N-k})(Y_{N-k} - i Y_k)
    const C2<T> ck = {mkk.x, -mkk.y}, cr = {mkr.x, -mkr.y};
    const C2<T> Wak = cmul(ck, C2<T>{Yak, -Yar}), Wbk = cmul(ck, C2<T>{Ybk, -Ybr});
    cb[j * ZS + k] = {Wak.x - Wbk.y, Wak.y + Wbk.x};
    if (k != 0 && kr != k) {
      const C2<T> War = cmul(cr, C2<T>{Yar, -Yak}), Wbr = cmul(cr, C2<T>{Ybr, -Ybk});
      cb[j * ZS + kr] = {War.x - Wbr.y, War.y + Wbr.x};
    }
  }
  __syncthreads();
  fft_core<T, N, KI>(lds, [&](int j, int n) { return cb[j * ZS + n]; }, tb);
  using O = OutItems<T, N, KI>;
  C2<T>* o = reinterpret_cast<C2<T>*>(field + a.base);
  const long ns = a.nstride / 2;
#pragma unroll 4
  for (int u = 0; u < O::PER_XY; ++u) {
    int j, k;
    if (O::xy(u, j, k)) {
      C2<T> v;
      post_pair<T, N, KI>(lds, tb, j, k, v.x, v.y);
      o[k * ns + j] = v;
    }
  }
}

// Register path of the same x pass, for R1 == R2 with one pass-2 task per thread.  The last
// forward radix pass leaves spectrum values k1 + R1 k2 (k2 < R2) of a job in the registers of
// the thread that owns k1, which is exactly the input set of the first inverse radix pass of
// stride R2 with n2 = k1: the weight is applied in registers and the transposes before and
// after it disappear.  The partner values at N - k are in the thread owning -k1 (mod R1); the
// pass-2 slots are ordered so that this thread is lane + 32 of the same wavefront (k1 = 0 and
// k1 = R1/2 hold their own partners), and the values are exchanged by lane shuffles.
template <int R1, int SW>
__device__ __forceinline__ int xmid_k1_of_slot(int slot) {
  constexpr int H = SW / 2;
  const int w = slot / SW, p = slot % SW;
  if (p < H) return w * H + p;
  const int kp = w * H + (p - H);
  return kp == 0 ? R1 / 2 : R1 - kp;
}

template <typename T, int N, int KF>
struct XmidRegs {
  using S = TileCfg<T, N, KF>;
  static constexpr int SW = 64 / S::NJ;  // pass-2 slots per wavefront
  static constexpr bool ok = S::R3 == 1 && S::R1 == S::R2 && S::NJ * S::R1 == S::NT && S::NJ * S::R2 == S::NT &&
                             S::NT % 64 == 0 && 64 % S::NJ == 0 && SW % 2 == 0 && S::R1 % SW == 0;
};

// LDS of the register-path x pass: the transform work area, then (float32) the tables the pass
// reads between its transforms: the pass twiddles tw[i] (i <= (M - 1)(R1 - 1), which covers the
// second-pass twiddles of three passes too), mk and the x eigenvalues of the block's component,
// copied once per block so that no table read waits behind the tile's outstanding sample loads.
// Only where the tables keep the resident blocks per compute unit; float64 blocks keep them in
// global memory (their larger entries would cost a resident block per compute unit).
template <typename T, int N, int KF>
struct XmidRegs3;
template <typename T, int N>
struct XmidLds {
  using S = TileCfg<T, N, DCT2>;
  static constexpr bool REGS = (XmidRegs<T, N, DCT2>::ok && XmidRegs<T, N, DST2>::ok) ||
                               (XmidRegs3<T, N, DCT2>::ok && XmidRegs3<T, N, DST2>::ok);
  static constexpr int NTW = (S::M - 1) * (S::R1 - 1) + 1;
  static constexpr size_t TAB_OFF = (S::BYTES + 15) / 16 * 16;
  static constexpr size_t TAB_BYTES = TAB_OFF + (size_t)(NTW + N) * sizeof(C2<T>) + (size_t)N * sizeof(T);
  static constexpr bool TABLES = REGS && sizeof(T) == 4 && 163840 / TAB_BYTES >= 163840 / S::BYTES;
  static constexpr size_t BYTES = TABLES ? TAB_BYTES : S::BYTES;
};

template <typename T, int N, int KF, int KI>
__device__ void xmid_tile_regs(T* lds, T* field, int tile, int mc, double mu, const Tab<T>& tb,
                               C2<T> (&zs)[TileCfg<T, N, KF>::PT1][TileCfg<T, N, KF>::R1], const T* lxt, T ly,
                               const T (&lz)[2]) {
  using S = TileCfg<T, N, KF>;
  constexpr int W = S::W, NJ = S::NJ, R1 = S::R1, R2 = S::R2, SW = XmidRegs<T, N, KF>::SW;
  static_assert(XmidRegs<T, N, KF>::ok, "register path needs R1 == R2 and one task per thread");
  const TileAddr a = tile_addr<W, N>(0, tile);
  C2<T>* cb = reinterpret_cast<C2<T>*>(lds);
  const int tid = threadIdx.x, j = tid % NJ;
  // forward: pass 1 of task (j, tid / NJ), then pass 2 of task (j, k1) in the paired slot order
  fft_pass1_dft<T, N, KF>(tid / NJ, zs[0], tb);
  fft_pass1_store<T, N, KF>(cb, zs[0], j, tid / NJ);
  __syncthreads();
  const int k1 = xmid_k1_of_slot<R1, SW>(tid / NJ);
  C2<T> z[R2];
  fft_pass2_dft<T, N, KF>(cb, z, j, k1);  // z[k2] = Z_k, k = k1 + R1 k2
  // Z_{N-k} is register R2 - 1 - k2 of the partner (k1 != 0) or of the thread itself
  // (k1 = R1/2), and register (R2 - k2) mod R2 of the thread itself for k1 = 0
  const int lane = tid & 63;
  const bool own = (k1 == 0) || (2 * k1 == R1);
  const int src = own ? lane : (lane ^ 32);
  const bool zero_k1 = (k1 == 0);
  const bool wave_has_zero = (tid / 64) == 0;  // slot 0 (k1 = 0) is in the first wavefront
  C2<T> zr[R2];
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    zr[k2].x = __shfl(z[R2 - 1 - k2].x, src, 64);
    zr[k2].y = __shfl(z[R2 - 1 - k2].y, src, 64);
  }
  if (wave_has_zero) {
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2)
      if (zero_k1) zr[k2] = z[(R2 - k2) & (R2 - 1)];
  }
  const T mu2 = T(2 * mu);  // the factor 1/2 of V is folded into the weight denominators
  T ya[R2], yb[R2];
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    const int k = k1 + R1 * k2;
    const int mode = (KF == DST2) ? N - 1 - k : k;
    const T lx = lxt[mode];
    T om[2];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const T num = (mc == 0) ? lx : (mc == 1) ? ly : lz[w];
      const T den = mu2 * (lx + ly + lz[w]);
      if constexpr (sizeof(T) == 4)
        om[w] = num * __builtin_amdgcn_rcpf(den);  // 1 ulp: the float32 inner solve
      else
        om[w] = num / den;
    }
    const C2<T> Zk = z[k2], Zr = zr[k2], mkk = tb.mk[k];
    const C2<T> Va = {Zk.x + Zr.x, Zk.y - Zr.y};  // 2 V^a_k
    const C2<T> Vb = {Zk.y + Zr.y, Zr.x - Zk.x};  // 2 V^b_k
    ya[k2] = om[0] * (mkk.x * Va.x - mkk.y * Va.y);
    yb[k2] = om[1] * (mkk.x * Vb.x - mkk.y * Vb.y);
  }
  // Y_{N-k} from the same place as Z_{N-k} (Y_N = 0)
  T yar[R2], ybr[R2];
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    yar[k2] = __shfl(ya[R2 - 1 - k2], src, 64);
    ybr[k2] = __shfl(yb[R2 - 1 - k2], src, 64);
  }
  if (wave_has_zero) {
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2)
      if (zero_k1) {
        yar[k2] = (k2 == 0) ? T(0) : ya[(R2 - k2) & (R2 - 1)];
        ybr[k2] = (k2 == 0) ? T(0) : yb[(R2 - k2) & (R2 - 1)];
      }
  }
  // inverse input Z'_k = V'^a_k + i V'^b_k, V'_k = conj(mk_k)(Y_k - i Y_{N-k})
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    const C2<T> mk = tb.mk[k1 + R1 * k2], ck = {mk.x, -mk.y};
    const C2<T> Wa = cmul(ck, C2<T>{ya[k2], -yar[k2]}), Wb = cmul(ck, C2<T>{yb[k2], -ybr[k2]});
    z[k2] = {Wa.x - Wb.y, Wa.y + Wb.x};
  }
  // inverse: pass 1 of task (j, n2 = k1) from registers, pass 2 in the natural order
  fft_pass1_dft<T, N, KI>(k1, z, tb);
  __syncthreads();  // the forward pass-2 reads of the transpose buffer are done
  fft_pass1_store<T, N, KI>(cb, z, j, k1);
  __syncthreads();
  fft_pass2_dft<T, N, KI>(cb, z, j, tid / NJ);
  __syncthreads();
  fft_pass2_store<T, N, KI>(cb, z, j, tid / NJ);
  __syncthreads();
  using O = OutItems<T, N, KI>;
  C2<T>* o = reinterpret_cast<C2<T>*>(field + a.base);
  const long ns = a.nstride / 2;
#pragma unroll
  for (int u = 0; u < O::PER_XY; ++u) {
    int jj, k;
    if (O::xy(u, jj, k)) {
      C2<T> v;
      post_pair<T, N, KI>(lds, tb, jj, k, v.x, v.y);
      o[k * ns + jj] = v;
    }
  }
}

// Register path of the x pass for three-pass transforms (R1 = R2 = R3 = 8, 32 threads per job).
// After the third forward pass a task (j, k1, k2) holds spectrum values k = k1 + 8 k2 + 64 k3
// (k3 < 8), exactly the input set of inverse pass-1 task m = k1 + 8 k2 (samples m + 64 n1).
// The partner values at N - k belong to task (8 - k1, 7 - k2) for k1 != 0 and (0, 8 - k2) for
// k1 = 0 (at k3' = 7 - k3), while (0, 0) (k3' = 8 - k3 mod 8) and (0, 4) (k3' = 7 - k3) are
// their own partners; every thread takes a task and its partner (slot 0 of a job takes (0, 0)
// and (0, 4)), so the weight is applied in registers without any lane exchange, and the
// spectrum transpose before it and the one after it disappear.
template <typename T, int N, int KF>
struct XmidRegs3 {
  using S = TileCfg<T, N, KF>;
  static constexpr bool ok = S::R1 == 8 && S::R2 == 8 && S::R3 == 8 && S::NT == S::NJ * 32;
};
// own ? a : b as a bitwise blend of the two values: a select between two register-array entries
// may otherwise be rewritten as a load through a selected address, which moves the arrays to
// scratch memory
template <typename T>
__device__ __forceinline__ T blend(uint32_t mask, T a, T b) {
  if constexpr (sizeof(T) == 4) {
    return __uint_as_float((__float_as_uint(a) & mask) | (__float_as_uint(b) & ~mask));
  } else {
    const uint64_t m = ((uint64_t)mask << 32) | mask;
    return __longlong_as_double((long long)(((uint64_t)__double_as_longlong(a) & m) |
                                            ((uint64_t)__double_as_longlong(b) & ~m)));
  }
}
template <typename T>
__device__ __forceinline__ C2<T> blend(uint32_t mask, C2<T> a, C2<T> b) {
  return {blend(mask, a.x, b.x), blend(mask, a.y, b.y)};
}

// the two pass-3 tasks (k1, k2) of pair slot p < 32 of a job
__device__ __forceinline__ void xmid3_tasks(int p, int& a1, int& a2, int& b1, int& b2) {
  if (p == 0) {
    a1 = 0, a2 = 0, b1 = 0, b2 = 4;
  } else if (p < 4) {
    a1 = 0, a2 = p, b1 = 0, b2 = 8 - p;
  } else {
    const int q = p - 4;  // 24 tasks with k1 = 1..3, then (4, 0..3)
    a1 = (q < 24) ? 1 + q / 8 : 4;
    a2 = (q < 24) ? q % 8 : q - 24;
    b1 = 8 - a1, b2 = 7 - a2;
  }
}

template <typename T, int N, int KF, int KI>
__device__ __forceinline__ void xmid_tile_regs3(T* lds, T* field, int tile, int mc, double mu, const Tab<T>& tb,
                                C2<T> (&zs)[TileCfg<T, N, KF>::PT1][TileCfg<T, N, KF>::R1], const T* lxt, T ly,
                                const T (&lz)[2]) {
  using S = TileCfg<T, N, KF>;
  constexpr int W = S::W, NJ = S::NJ;
  static_assert(XmidRegs3<T, N, KF>::ok && XmidRegs3<T, N, KI>::ok, "three radix-8 passes, two tasks per thread");
  const TileAddr a = tile_addr<W, N>(0, tile);
  C2<T>* cb = reinterpret_cast<C2<T>*>(lds);
  fft_pass1_all<T, N, KF>(cb, zs, tb);
  fft3_pass2<T, N, KF>(cb, tb);
  const int j = threadIdx.x % NJ, p = threadIdx.x / NJ;
  int a1, a2, b1, b2;
  xmid3_tasks(p, a1, a2, b1, b2);
  const uint32_t own = (p == 0) ? ~0u : 0u;  // tasks (0, 0) and (0, 4): partners inside each task
  C2<T> za[8], zb[8];
  fft3_pass3_task<T, N, KF>(cb, za, j, a1, a2);
  fft3_pass3_task<T, N, KF>(cb, zb, j, b1, b2);
  // Z_{N-k} for the values of task a and of task b
  C2<T> ra[8], rb[8];
#pragma unroll
  for (int k3 = 0; k3 < 8; ++k3) {
    ra[k3] = blend(own, za[(8 - k3) & 7], zb[7 - k3]);
    rb[k3] = blend(own, zb[7 - k3], za[7 - k3]);
  }
  const T mu2 = T(2 * mu);  // the factor 1/2 of V is folded into the weight denominators
  // Y_k of pencils a and b for the eight values of one task (k = k0 + 64 k3)
  auto weigh = [&](const C2<T>(&z)[8], const C2<T>(&r)[8], int k0, T(&ya)[8], T(&yb)[8]) {
#pragma unroll
    for (int k3 = 0; k3 < 8; ++k3) {
      const int k = k0 + 64 * k3;
      const int mode = (KF == DST2) ? N - 1 - k : k;
      const T lx = lxt[mode];
      T om[2];
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const T num = (mc == 0) ? lx : (mc == 1) ? ly : lz[w];
        const T den = mu2 * (lx + ly + lz[w]);
        if constexpr (sizeof(T) == 4)
          om[w] = num * __builtin_amdgcn_rcpf(den);  // 1 ulp: the float32 inner solve
        else
          om[w] = num / den;
      }
      const C2<T> Zk = z[k3], Zr = r[k3], mkk = tb.mk[k];
      const C2<T> Va = {Zk.x + Zr.x, Zk.y - Zr.y};  // 2 V^a_k
      const C2<T> Vb = {Zk.y + Zr.y, Zr.x - Zk.x};  // 2 V^b_k
      ya[k3] = om[0] * (mkk.x * Va.x - mkk.y * Va.y);
      yb[k3] = om[1] * (mkk.x * Vb.x - mkk.y * Vb.y);
    }
  };
  const int ka = a1 + 8 * a2, kb = b1 + 8 * b2;
  T yaa[8], yba[8], yab[8], ybb[8];  // y<pencil><task>
  weigh(za, ra, ka, yaa, yba);
  weigh(zb, rb, kb, yab, ybb);
  // inverse input Z'_k = V'^a_k + i V'^b_k, V'_k = conj(mk_k)(Y_k - i Y_{N-k}), Y_N = 0; the
  // Y_{N-k} sit where Z_{N-k} did
  auto prep = [&](const T(&ya)[8], const T(&yb)[8], const T(&yar)[8], const T(&ybr)[8], int k0, C2<T>(&z)[8]) {
#pragma unroll
    for (int k3 = 0; k3 < 8; ++k3) {
      const C2<T> mk = tb.mk[k0 + 64 * k3], ck = {mk.x, -mk.y};
      const C2<T> Wa = cmul(ck, C2<T>{ya[k3], -yar[k3]}), Wb = cmul(ck, C2<T>{yb[k3], -ybr[k3]});
      z[k3] = {Wa.x - Wb.y, Wa.y + Wb.x};
    }
  };
  T raa[8], rba[8], rab[8], rbb[8];
#pragma unroll
  for (int k3 = 0; k3 < 8; ++k3) {
    raa[k3] = blend(own, (k3 == 0) ? T(0) : yaa[(8 - k3) & 7], yab[7 - k3]);
    rba[k3] = blend(own, (k3 == 0) ? T(0) : yba[(8 - k3) & 7], ybb[7 - k3]);
    rab[k3] = blend(own, yab[7 - k3], yaa[7 - k3]);
    rbb[k3] = blend(own, ybb[7 - k3], yba[7 - k3]);
  }
  prep(yaa, yba, raa, rba, ka, za);
  prep(yab, ybb, rab, rbb, kb, zb);
  // inverse pass 1 of tasks m = k1 + 8 k2 from registers, then passes 2 and 3 from LDS
  fft_pass1_dft<T, N, KI>(ka, za, tb);
  fft_pass1_dft<T, N, KI>(kb, zb, tb);
  __syncthreads();  // every forward pass-3 read of the transpose buffer is done
  fft_pass1_store<T, N, KI>(cb, za, j, ka);
  fft_pass1_store<T, N, KI>(cb, zb, j, kb);
  __syncthreads();
  fft3_pass2<T, N, KI>(cb, tb);
  fft3_pass3<T, N, KI>(cb);
  using O = OutItems<T, N, KI>;
  C2<T>* o = reinterpret_cast<C2<T>*>(field + a.base);
  const long ns = a.nstride / 2;
#pragma unroll
  for (int u = 0; u < O::PER_XY; ++u) {
    int jj, k;
    if (O::xy(u, jj, k)) {
      C2<T> v;
      post_pair<T, N, KI>(lds, tb, jj, k, v.x, v.y);
      o[k * ns + jj] = v;
    }
  }
}

template <typename T, int N, int KIND>
__device__ __forceinline__ void store_xy_outputs(const T* lds, const Tab<T>& tb, T* out, long nstride) {
  using O = OutItems<T, N, KIND>;
  C2<T>* o = reinterpret_cast<C2<T>*>(out);
  const long ns = nstride / 2;
  // all outputs unrolled up to N = 256 (the pipelined forward y pair at 512 would spill)
  constexpr int UNROLL = N >= 512 ? 4 : O::PER_XY;
#pragma unroll UNROLL
  for (int u = 0; u < O::PER_XY; ++u) {
    int j, k;
    if (O::xy(u, j, k)) {
      C2<T> v;
      post_pair<T, N, KIND>(lds, tb, j, k, v.x, v.y);
      o[k * ns + j] = v;
    }
  }
}

// ---------------------------------------------------------------------------------------
// fused x pass of the right-hand side and of the velocity back-substitution, component m:
//   RHS      (KF = T_m along x, KI = C_m^T along x): fh = KF(in) (the full T_m F_m, kept for
//            the back-substitution), out = KI(-sigma_m / (mu Lambda_m) fh)
//   BACKSUB  (KF = C_m along x, KI = T_m^T along x): out = KI((fh + sigma_m KF(in)) / (mu Lambda_m))
// The forward outputs go to registers, are weighted (and fh read or written), and the tile
// is restaged in LDS for the inverse.
// ---------------------------------------------------------------------------------------
// LDS of the fused x passes of the right-hand side and the back-substitution: the transform
// work area, then (float32, where the resident blocks per compute unit stay the same) the
// tables read between the transforms: the twiddles of the two kinds (one table when their
// lengths agree), mk and the x eigenvalues of the component.
template <typename T, int N, int KF, int KI>
struct XfuseLds {
  using SF = TileCfg<T, N, KF>;
  using SI = TileCfg<T, N, KI>;
  static constexpr size_t WORK = SF::BYTES > SI::BYTES ? SF::BYTES : SI::BYTES;
  static constexpr size_t TAB_OFF = (WORK + 15) / 16 * 16;
  static constexpr bool SHARE = SF::L == SI::L;
  static constexpr int NTW = SF::L + (SHARE ? 0 : SI::L);
  static constexpr size_t TAB_BYTES = TAB_OFF + (size_t)(NTW + N) * sizeof(C2<T>) + (size_t)N * sizeof(T);
  static constexpr bool ON = sizeof(T) == 4 && 163840 / TAB_BYTES >= 163840 / WORK;
  static constexpr size_t BYTES = ON ? TAB_BYTES : WORK;
};

template <typename T, int N, int KF, int KI, bool BACKSUB>
__global__ __launch_bounds__(tile_nt_max<N>()) __attribute__((amdgpu_waves_per_eu(xfuse_waves<T, N>()))) void k_xfuse(const T* __restrict__ in, T* __restrict__ fh, T* __restrict__ out,
                                              int m, double mu, Tab<T> tb, Bat bt) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (rhs_skipped(bt)) return;
  in = wb(in, bt);
  fh = wb(fh, bt);
  out = wb(out, bt);
  T* lds = reinterpret_cast<T*>(smem);
  using SF = TileCfg<T, N, KF>;
  using SI = TileCfg<T, N, KI>;
  using OF = OutItems<T, N, KF>;
  using X = XfuseLds<T, N, KF, KI>;
  static_assert(SF::W == SI::W, "one tile for both transforms");
  static_assert(KF == DCT2 || KF == DST2 || KF == DST1, "the forward kind gathers without tables");
  constexpr int W = SF::W, RS = N + 1, NT = SF::NT;
  const TileAddr a = tile_addr<W, N>(0, blockIdx.x);
  const int yi = blockIdx.x / (N / W), z0 = (blockIdx.x % (N / W)) * W, j0 = threadIdx.x % SF::NJ;
  // sigma_m^2 / Lambda_m parts: y and z eigenvalues of the thread's pencils (z indices z0 + 2 j0,
  // z0 + 2 j0 + 1, the same for all its outputs), and sigma_m where m is not x; the index along
  // m is mode k of the DCT-II / DST-I, along the other axes mode k + 1 of the DST-II
  // (read before the samples where the tables go to LDS, after the transform otherwise, which
  // keeps them out of the float64 kernels' register peak)
  const T* gx = (m == 0) ? tb.sg2 : tb.sg2s;
  T ly, lz[2], sgc[2];
  auto load_parts = [&]() {
    ly = (m == 1) ? tb.sg2[yi] : tb.sg2s[yi];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const int iz = z0 + 2 * j0 + w;
      lz[w] = (m == 2) ? tb.sg2[iz] : tb.sg2s[iz];
      const T sq = (m == 1) ? tb.sg2[yi] : (m == 2) ? tb.sg2[iz] : T(1);
      if constexpr (sizeof(T) == 4)
        sgc[w] = __builtin_sqrtf(sq);
      else
        sgc[w] = sqrt(sq);
    }
  };
  if constexpr (X::ON) load_parts();
  // tables requested before the samples (published to LDS once they have arrived)
  constexpr int PLF = X::ON ? (SF::L + NT - 1) / NT : 1, PLI = (X::ON && !X::SHARE) ? (SI::L + NT - 1) / NT : 1;
  constexpr int PN = X::ON ? (N + NT - 1) / NT : 1;
  C2<T> rtf[PLF], rti[PLI], rmk[PN];
  T rgx[PN];
  const C2<T>* gtf = (SF::L == N) ? tb.tw : tb.tw2;
  const C2<T>* gti = (SI::L == N) ? tb.tw : tb.tw2;
  if constexpr (X::ON) {
#pragma unroll
    for (int u = 0; u < PLF; ++u) {
      const int i = threadIdx.x + u * NT;
      if (i < SF::L) rtf[u] = gtf[i];
    }
    if constexpr (!X::SHARE) {
#pragma unroll
      for (int u = 0; u < PLI; ++u) {
        const int i = threadIdx.x + u * NT;
        if (i < SI::L) rti[u] = gti[i];
      }
    }
#pragma unroll
    for (int u = 0; u < PN; ++u) {
      const int i = threadIdx.x + u * NT;
      if (i < N) {
        rmk[u] = tb.mk[i];
        rgx[u] = gx[i];
      }
    }
  }
  C2<T>* fp = reinterpret_cast<C2<T>*>(fh + a.base);
  const long ns = a.nstride / 2;
  C2<T> f[BACKSUB ? OF::PER_XY : 1];
  if constexpr (BACKSUB) {
#pragma unroll
    for (int u = 0; u < OF::PER_XY; ++u) {
      int j, k;
      if (OF::xy(u, j, k)) f[u] = fp[k * ns + j];
    }
  }
  const GlobSrc<T> src{in, a.base, a.nstride};
  Tab<T> tl = tb;
  const T* lgx = gx;
  if constexpr (X::ON) {
    C2<T> z[SF::PT1][SF::R1];
    fft_gather<T, N, KF>([&](int j, int n) { return pre_sample<T, N, KF>(src, tb, j, n); }, z);
    C2<T>* ltf = reinterpret_cast<C2<T>*>(smem + X::TAB_OFF);
    C2<T>* lti = X::SHARE ? ltf : ltf + SF::L;
    C2<T>* lmk = ltf + X::NTW;
    T* lg = reinterpret_cast<T*>(lmk + N);
#pragma unroll
    for (int u = 0; u < PLF; ++u) {
      const int i = threadIdx.x + u * NT;
      if (i < SF::L) ltf[i] = rtf[u];
    }
    if constexpr (!X::SHARE) {
#pragma unroll
      for (int u = 0; u < PLI; ++u) {
        const int i = threadIdx.x + u * NT;
        if (i < SI::L) lti[i] = rti[u];
      }
    }
#pragma unroll
    for (int u = 0; u < PN; ++u) {
      const int i = threadIdx.x + u * NT;
      if (i < N) {
        lmk[i] = rmk[u];
        lg[i] = rgx[u];
      }
    }
    if (SF::L == N) tl.tw = ltf; else tl.tw2 = ltf;
    if (SI::L == N) tl.tw = lti; else tl.tw2 = lti;
    tl.mk = lmk;
    lgx = lg;
    __syncthreads();
    fft_core_from<T, N, KF>(lds, z, tl);
  } else {
    fft_tile<T, N, KF>(lds, src, tb);
    load_parts();
  }
  C2<T> v[OF::PER_XY];
#pragma unroll
  for (int u = 0; u < OF::PER_XY; ++u) {
    int j, k;
    if (OF::xy(u, j, k)) {
      post_pair<T, N, KF>(lds, tl, j, k, v[u].x, v[u].y);
      // sigma_m and 1 / (mu Lambda_m) of the two pencils
      const T lx = lgx[k];
      T sg[2], il[2];
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const T lam = lx + ly + lz[w];
        if constexpr (sizeof(T) == 4) {
          sg[w] = (m == 0) ? __builtin_sqrtf(lx) : sgc[w];
          il[w] = __builtin_amdgcn_rcpf(T(mu) * lam);  // 1 ulp: the float32 inner solve
        } else {
          sg[w] = (m == 0) ? sqrt(lx) : sgc[w];
          il[w] = T(1) / (T(mu) * lam);
        }
      }
      if constexpr (BACKSUB) {
        v[u].x = (f[u].x + sg[0] * v[u].x) * il[0];
        v[u].y = (f[u].y + sg[1] * v[u].y) * il[1];
      } else {
        fp[k * ns + j] = v[u];
        v[u].x = -sg[0] * il[0] * v[u].x;
        v[u].y = -sg[1] * il[1] * v[u].y;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < OF::PER_XY; ++u) {
    int j, k;
    if (OF::xy(u, j, k)) {
      lds[(2 * j) * RS + k] = v[u].x;
      lds[(2 * j + 1) * RS + k] = v[u].y;
    }
  }
  __syncthreads();
  fft_tile<T, N, KI>(lds, LdsSrc<T, N>{lds}, tl);
  store_xy_outputs<T, N, KI>(lds, tl, out + a.base, a.nstride);
}

// one tile per block (two tiles per block, with the second tile's samples requested before the
// first is transformed, measured slower: 125 vs 118 us at 256^3 float32)
template <typename T, int N, int KF, int KI>
__device__ void xmid_body(T* lds, T* field, int mc, double mu, const Tab<T>& tb) {
  using S = TileCfg<T, N, KF>;
  const int tile = blockIdx.x;
  const TileAddr a = tile_addr<S::W, N>(0, tile);
  const GlobSrc<T> src{field, a.base, a.nstride};
  C2<T> zs[S::PT1][S::R1];
  using X = XmidLds<T, N>;
  if constexpr (X::REGS) {
    constexpr bool THREE = XmidRegs3<T, N, KF>::ok;
    auto run = [&](const Tab<T>& t, const T* lxt, T ly, const T(&lz)[2]) {
      if constexpr (THREE)
        xmid_tile_regs3<T, N, KF, KI>(lds, field, tile, mc, mu, t, zs, lxt, ly, lz);
      else
        xmid_tile_regs<T, N, KF, KI>(lds, field, tile, mc, mu, t, zs, lxt, ly, lz);
    };
    // y and z eigenvalues of the thread's two pencils, the x eigenvalues of the component
    const int yi = tile / (N / S::W), z0 = (tile % (N / S::W)) * S::W, j = threadIdx.x % S::NJ;
    const T ly = (mc == 1) ? tb.sg2[yi] : tb.sg2s[yi];
    T lz[2];
#pragma unroll
    for (int w = 0; w < 2; ++w) lz[w] = (mc == 2) ? tb.sg2[z0 + 2 * j + w] : tb.sg2s[z0 + 2 * j + w];
    const T* gx = (mc == 0) ? tb.sg2 : tb.sg2s;
    if constexpr (X::TABLES) {
      // table entries requested before the samples, written to LDS once they (not the samples) are in
      constexpr int NT = S::NT, PT = (X::NTW + NT - 1) / NT, PN = (N + NT - 1) / NT;
      unsigned char* base = reinterpret_cast<unsigned char*>(lds) + X::TAB_OFF;
      C2<T>* ltw = reinterpret_cast<C2<T>*>(base);
      C2<T>* lmk = ltw + X::NTW;
      T* lsg = reinterpret_cast<T*>(lmk + N);
      C2<T> rtw[PT], rmk[PN];
      T rsg[PN];
#pragma unroll
      for (int u = 0; u < PT; ++u) {
        const int i = threadIdx.x + u * NT;
        if (i < X::NTW) rtw[u] = tb.tw[i];
      }
#pragma unroll
      for (int u = 0; u < PN; ++u) {
        const int i = threadIdx.x + u * NT;
        if (i < N) {
          rmk[u] = tb.mk[i];
          rsg[u] = gx[i];
        }
      }
      fft_gather<T, N, KF>([&](int jj, int n) { return pre_sample<T, N, KF>(src, tb, jj, n); }, zs);
#pragma unroll
      for (int u = 0; u < PT; ++u) {
        const int i = threadIdx.x + u * NT;
        if (i < X::NTW) ltw[i] = rtw[u];
      }
#pragma unroll
      for (int u = 0; u < PN; ++u) {
        const int i = threadIdx.x + u * NT;
        if (i < N) {
          lmk[i] = rmk[u];
          lsg[i] = rsg[u];
        }
      }
      __syncthreads();
      Tab<T> tl = tb;
      tl.tw = ltw;
      tl.mk = lmk;
      run(tl, lsg, ly, lz);
    } else {
      fft_gather<T, N, KF>([&](int jj, int n) { return pre_sample<T, N, KF>(src, tb, jj, n); }, zs);
      run(tb, gx, ly, lz);
    }
  } else {
    fft_gather<T, N, KF>([&](int j, int n) { return pre_sample<T, N, KF>(src, tb, j, n); }, zs);
    xmid_tile<T, N, KF, KI>(lds, field, tile, mc, mu, tb, zs);
  }
}

template <typename T, int N>
__global__ __launch_bounds__(tile_nt_max<N>()) void k_xmid(T* A0, T* A1, T* A2, double mu, Tab<T> tb, Bat bt) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (rhs_skipped(bt)) return;
  A0 = wb(A0, bt);
  A1 = wb(A1, bt);
  A2 = wb(A2, bt);
  T* lds = reinterpret_cast<T*>(smem);
  // float64: the component written last by the y passes (2) first, while it is still in the
  // last-level cache (27.6 -> 26.9 ms per float64 evaluation at 256^3, the following inverse y
  // pass gaining as well); float32 measured slightly better in the natural order
  const int mc = (sizeof(T) == 8) ? 2 - (int)blockIdx.y : (int)blockIdx.y;
  if (mc == 0)
    xmid_body<T, N, DCT2, DCT3>(lds, A0, 0, mu, tb);
  else if (mc == 1)
    xmid_body<T, N, DST2, DST3>(lds, A1, 1, mu, tb);
  else
    xmid_body<T, N, DST2, DST3>(lds, A2, 2, mu, tb);
}


// ---------------------------------------------------------------------------------------
// CG z-passes with fused vector updates
// ---------------------------------------------------------------------------------------
// d = r + beta d_old (written back), A = DST-II_z(d), B = DCT-II_z(d): one read of r and d
// for both transforms (the tile is restaged in LDS from registers for the second)
template <typename T, int N, int KIND>
__device__ __forceinline__ void store_z_outputs(const T* lds, const Tab<T>& tb, T* out) {
  using O = OutItems<T, N, KIND>;
  V16<T>* o = reinterpret_cast<V16<T>*>(out);
  constexpr int RV = N / O::VEC;
#pragma unroll
  for (int u = 0; u < O::PER_Z; ++u) {
    int j, k0;
    if (O::z(u, j, k0)) {
      V16<T> v0, v1;
      O::z_values(lds, tb, j, k0, v0, v1);
      o[(2 * j) * RV + k0 / O::VEC] = v0;
      o[(2 * j + 1) * RV + k0 / O::VEC] = v1;
    }
  }
}

// Forward z pass of the Schur matvec with the CG vector updates folded in.
//   ZF_PLAIN  A = DST-II_z r, B = DCT-II_z r (velocity back-substitution; r is only read)
//   ZF_FIRST  r -= mean r (the mean from the sum in scal[9]), d = r, x = 0, then the transforms of
//             d; partial sums of r.r
//   ZF_FUSED  x += alpha d, r -= alpha (q - mean q), d = r + beta d (alpha, beta, mean q of the
//             previous iteration in scal[1..3]), then the transforms of d; partial sums of r.r
//   ZF_FINAL  r += alpha d (the pending update of the CG iterate, r = x), written back, then its
//             transforms (velocity back-substitution)
// Every thread streams its vectors once; d stays in registers for the second transform.
template <typename T, int N, int MODE>
__global__ __launch_bounds__(tile_nt_max<N>()) void k_zfwd_cg(T* __restrict__ x, T* __restrict__ r, T* __restrict__ d,
                                                const T* __restrict__ q, T* __restrict__ A, T* __restrict__ B,
                                                const double* __restrict__ scal, double* __restrict__ rpart,
                                                Tab<T> tg, Bat bt) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[tile_nt_max<N>() / 64];
  if (rhs_skipped(bt)) return;
  x = wb(x, bt);
  r = wb(r, bt);
  d = wb(d, bt);
  q = wb(q, bt);
  A = wb(A, bt);
  B = wb(B, bt);
  scal = wb(scal, bt);
  rpart = wb(rpart, bt);
  T* lds = reinterpret_cast<T*>(smem);
  using S = TileCfg<T, N, DST2>;
  constexpr int W = S::W, RS = N + 1, NT = S::NT, VEC = V16<T>::n;
  constexpr int NV = W * N / VEC, PER = (NV + NT - 1) / NT;
  const TileAddr a = tile_addr<W, N>(2, blockIdx.x);
  TabStage<T, N, DST2> ts;  // DST-II and DCT-II read the same tables
  ts.request(tg);
  const V16<T>* rv = reinterpret_cast<const V16<T>*>(r + a.base);
  V16<T> v[PER];
  double rr = 0;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = threadIdx.x + u * NT;
    if (NV % NT == 0 || e < NV) {
      v[u] = rv[e];
      if constexpr (MODE == ZF_FUSED) {
        const T alpha = T(scal[1]), beta = T(scal[2]), mq = T(scal[3]);
        V16<T>* xv = reinterpret_cast<V16<T>*>(x + a.base);
        V16<T>* wv = reinterpret_cast<V16<T>*>(r + a.base);
        V16<T>* dv = reinterpret_cast<V16<T>*>(d + a.base);
        const V16<T> dold = dv[e], qv = reinterpret_cast<const V16<T>*>(q + a.base)[e];
        V16<T> xn = xv[e];
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
          xn.a[c] += alpha * dold.a[c];
          v[u].a[c] -= alpha * (qv.a[c] - mq);
        }
        xv[e] = xn;
        wv[e] = v[u];
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
          rr += (double)v[u].a[c] * (double)v[u].a[c];
          v[u].a[c] += beta * dold.a[c];
        }
        dv[e] = v[u];
      } else if constexpr (MODE == ZF_FINAL) {
        const T alpha = T(scal[1]);
        const V16<T> dv = reinterpret_cast<const V16<T>*>(d + a.base)[e];
#pragma unroll
        for (int c = 0; c < VEC; ++c) v[u].a[c] += alpha * dv.a[c];
        reinterpret_cast<V16<T>*>(r + a.base)[e] = v[u];
      } else if constexpr (MODE == ZF_FIRST) {
        const T shift = T(scal[9] * (-1.0 / ((double)N * N * N)));
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
          v[u].a[c] += shift;
          rr += (double)v[u].a[c] * (double)v[u].a[c];
        }
        V16<T> zero;
#pragma unroll
        for (int c = 0; c < VEC; ++c) zero.a[c] = T(0);
        reinterpret_cast<V16<T>*>(r + a.base)[e] = v[u];
        reinterpret_cast<V16<T>*>(d + a.base)[e] = v[u];
        reinterpret_cast<V16<T>*>(x + a.base)[e] = zero;
      }
    }
  }
  const Tab<T> tb = ts.publish(smem, tg);  // read after the first stage's barrier
  if constexpr (MODE == ZF_FIRST || MODE == ZF_FUSED) {
    const double t = block_sum(rr, red);
    if (threadIdx.x == 0) rpart[blockIdx.x] = t;
  }
  auto stage = [&]() {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = threadIdx.x + u * NT;
      if (NV % NT == 0 || e < NV) {
        const int p = (e * VEC) / N, n = (e * VEC) - p * N;
#pragma unroll
        for (int c = 0; c < VEC; ++c) lds[p * RS + n + c] = v[u].a[c];
      }
    }
    __syncthreads();
  };
  stage();
  fft_tile<T, N, DST2>(lds, LdsSrc<T, N>{lds}, tb);
  store_z_outputs<T, N, DST2>(lds, tb, A + a.base);
  __syncthreads();
  stage();
  fft_tile<T, N, DCT2>(lds, LdsSrc<T, N>{lds}, tb);
  store_z_outputs<T, N, DCT2>(lds, tb, B + a.base);
}

// q = DST-III_z(A) + DCT-III_z(B) + c d; per-block partial sums of d.q, q, d, q.q
template <typename T, int N>
__global__ __launch_bounds__(tile_nt_max<N>()) __attribute__((amdgpu_waves_per_eu(tile_waves<T, N>()))) void k_zinv_cg(const T* __restrict__ A, const T* __restrict__ B,
                                                T* __restrict__ q, const T* __restrict__ d, double c,
                                                double* __restrict__ partials, Tab<T> tg, Bat bt) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[4 * (tile_nt_max<N>() / 64)];  // 4 sums per wavefront
  if (rhs_skipped(bt)) return;
  A = wb(A, bt);
  B = wb(B, bt);
  q = wb(q, bt);
  d = wb(d, bt);
  partials = wb(partials, bt);
  T* lds = reinterpret_cast<T*>(smem);
  using S = TileCfg<T, N, DCT3>;
  using O = OutItems<T, N, DCT3>;
  constexpr int W = S::W, NT = S::NT, VEC = V16<T>::n, RV = N / VEC;
  const TileAddr a = tile_addr<W, N>(2, blockIdx.x);
  // tables, then the A tile, then the B tile (staged in LDS after the first transform) are
  // requested; the tables and the A tile go to LDS as they arrive
  using TS = TabStage<T, N, DST3>;
  TS ts;
  ts.request(tg);
  constexpr int NV = W * N / VEC, PV = (NV + NT - 1) / NT;
  V16<T> vb[PV];
  if constexpr (TS::ON) {
    V16<T> va[PV];
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int e = threadIdx.x + u * NT;
      if (NV % NT == 0 || e < NV) va[u] = reinterpret_cast<const V16<T>*>(A + a.base)[e];
    }
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int e = threadIdx.x + u * NT;
      if (NV % NT == 0 || e < NV) vb[u] = reinterpret_cast<const V16<T>*>(B + a.base)[e];
    }
    (void)ts.publish(smem, tg);
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int e = threadIdx.x + u * NT;
      if (NV % NT == 0 || e < NV) {
        const int p = (e * VEC) / N, n = (e * VEC) - p * N;
#pragma unroll
        for (int qq = 0; qq < VEC; ++qq) lds[p * (N + 1) + n + qq] = va[u].a[qq];
      }
    }
    __syncthreads();
  } else {  // float64: the A tile is staged before the B tile is requested (register budget)
    load_tile_z<T, N, NT>(lds, A + a.base);
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int e = threadIdx.x + u * NT;
      if (NV % NT == 0 || e < NV) vb[u] = reinterpret_cast<const V16<T>*>(B + a.base)[e];
    }
  }
  const Tab<T> tb = TS::view(smem, tg);
  fft_tile<T, N, DST3>(lds, LdsSrc<T, N>{lds}, tb);
  V16<T> acc[2 * O::PER_Z];
#pragma unroll
  for (int u = 0; u < O::PER_Z; ++u) {
    int j, k0;
    if (O::z(u, j, k0)) OutItems<T, N, DST3>::z_values(lds, tb, j, k0, acc[2 * u], acc[2 * u + 1]);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PV; ++u) {
    const int e = threadIdx.x + u * NT;
    if (NV % NT == 0 || e < NV) {
      const int p = (e * VEC) / N, n = (e * VEC) - p * N;
#pragma unroll
      for (int qq = 0; qq < VEC; ++qq) lds[p * (N + 1) + n + qq] = vb[u].a[qq];
    }
  }
  __syncthreads();
  // the d vectors of the thread are requested before the second transform
  const V16<T>* dv = reinterpret_cast<const V16<T>*>(d + a.base);
  V16<T> dd[2 * O::PER_Z];
#pragma unroll
  for (int u = 0; u < O::PER_Z; ++u) {
    int j, k0;
    if (O::z(u, j, k0)) {
      dd[2 * u] = dv[(2 * j) * RV + k0 / VEC];
      dd[2 * u + 1] = dv[(2 * j + 1) * RV + k0 / VEC];
    }
  }
  fft_tile<T, N, DCT3>(lds, LdsSrc<T, N>{lds}, tb);
  V16<T>* qv = reinterpret_cast<V16<T>*>(q + a.base);
  double sdq = 0, sq = 0, sd = 0, sqq = 0;
  const T cc = T(c);
#pragma unroll
  for (int u = 0; u < O::PER_Z; ++u) {
    int j, k0;
    if (O::z(u, j, k0)) {
      V16<T> v[2];
      O::z_values(lds, tb, j, k0, v[0], v[1]);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const T dvv = dd[2 * u + h].a[e];
          const T qn = acc[2 * u + h].a[e] + v[h].a[e] + cc * dvv;
          v[h].a[e] = qn;
          sdq += (double)dvv * (double)qn;
          sqq += (double)qn * (double)qn;
          sq += (double)qn;
          sd += (double)dvv;
        }
        qv[(2 * j + h) * RV + k0 / VEC] = v[h];
      }
    }
  }
  double t[4] = {sdq, sq, sd, sqq};
  block_sum4(t, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) partials[4 * blockIdx.x + c] = t[c];
}

template <typename T, int N>
__device__ __forceinline__ void ypair_fwd_body(T* lds, const T* __restrict__ A, T* __restrict__ A1, T* __restrict__ B2,
                                               const Tab<T>& tg, int blk) {
  using S = TileCfg<T, N, DCT2>;
  static_assert(S::R1 == TileCfg<T, N, DST2>::R1 && S::M == TileCfg<T, N, DST2>::M, "one gather for both kinds");
  constexpr int W = S::W, R1 = S::R1;
  const TileAddr a = tile_addr<W, N>(1, blk);
  const GlobSrc<T> src{A, a.base, a.nstride};
  TabStage<T, N, DCT2> ts;  // DCT-II and DST-II read the same tables
  ts.request(tg);
  C2<T> zc[S::PT1][R1], zs[S::PT1][R1];
  fft_gather<T, N, DCT2>([&](int j, int n) { return pre_sample<T, N, DCT2>(src, tg, j, n); }, zc);
  const Tab<T> tb = ts.publish(reinterpret_cast<unsigned char*>(lds), tg);
  if constexpr (TabStage<T, N, DCT2>::ON) __syncthreads();
#pragma unroll
  for (int u = 0; u < S::PT1; ++u)
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) {
      // sample M n1 + m (m < M) comes from an odd source index iff M n1 + m >= N/2
      static_assert((N / 2) % S::M == 0, "the sign of a sample depends on n1 only");
      const bool odd = S::M * n1 >= N / 2;
      zs[u][n1] = odd ? C2<T>{-zc[u][n1].x, -zc[u][n1].y} : zc[u][n1];
    }
  fft_core_from<T, N, DST2>(lds, zs, tb);
  store_xy_outputs<T, N, DST2>(lds, tb, A1 + a.base, a.nstride);
  fft_core_from<T, N, DCT2>(lds, zc, tb);
  store_xy_outputs<T, N, DCT2>(lds, tb, B2 + a.base, a.nstride);
}

template <typename T, int N>
__device__ __forceinline__ void ypair_inv_body(T* lds, const T* __restrict__ A1, const T* __restrict__ B2,
                                               T* __restrict__ A, const Tab<T>& tb, int blk) {
  using O = OutItems<T, N, DST3>;
  constexpr int W = TileCfg<T, N, DST3>::W;
  const TileAddr a = tile_addr<W, N>(1, blk);
  fft_tile<T, N, DST3>(lds, GlobSrc<T>{A1, a.base, a.nstride}, tb);
  C2<T> acc[O::PER_XY];
#pragma unroll
  for (int u = 0; u < O::PER_XY; ++u) {
    int j, k;
    if (O::xy(u, j, k)) post_pair<T, N, DST3>(lds, tb, j, k, acc[u].x, acc[u].y);
  }
  fft_tile<T, N, DCT3>(lds, GlobSrc<T>{B2, a.base, a.nstride}, tb);
  C2<T>* o = reinterpret_cast<C2<T>*>(A + a.base);
  const long ns = a.nstride / 2;
#pragma unroll
  for (int u = 0; u < O::PER_XY; ++u) {
    int j, k;
    if (O::xy(u, j, k)) {
      C2<T> v;
      post_pair<T, N, DCT3>(lds, tb, j, k, v.x, v.y);
      v.x += acc[u].x;
      v.y += acc[u].y;
      o[k * ns + j] = v;
    }
  }
}

// y passes of the Schur matvec with two transforms per block.
// forward: A1 = DST-II_y(A), B2 = DCT-II_y(A); inverse: A = DST-III_y(A1) + DCT-III_y(B2)
// The DST-II input is the DCT-II input (Makhoul order) with the samples from the second half of
// the reordered pencil negated: one gather serves both transforms, A is read once.
template <typename T, int N>
__global__ __launch_bounds__(tile_nt_max<N>()) void k_ypair_fwd(const T* __restrict__ A, T* __restrict__ A1, T* __restrict__ B2,
                                                  Tab<T> tb, Bat bt) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (rhs_skipped(bt)) return;
  ypair_fwd_body<T, N>(reinterpret_cast<T*>(smem), wb(A, bt), wb(A1, bt), wb(B2, bt), tb, blockIdx.x);
}

template <typename T, int N>
__global__ __launch_bounds__(tile_nt_max<N>()) void k_ypair_inv(const T* __restrict__ A1, const T* __restrict__ B2,
                                                  T* __restrict__ A, Tab<T> tb, Bat bt) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (rhs_skipped(bt)) return;
  ypair_inv_body<T, N>(reinterpret_cast<T*>(smem), wb(A1, bt), wb(B2, bt), wb(A, bt), tb, blockIdx.x);
}


// Persistent, pipelined form of the forward y pair: the raw rows of the block's tile are staged
// in LDS, the rows of its next tile are requested into registers, and the pass-1 samples of both
// transforms come from one gather of the staged rows (the DST-II input being the DCT-II input
// with sign flips); tables (twiddles, mk, s_k, shared by the two kinds) in LDS.
template <typename T, int N>
__global__ __launch_bounds__(tile_nt_max<N>()) void k_ypair_fwd_pipe(const T* __restrict__ A, T* __restrict__ A1,
                                                       T* __restrict__ B2, int ntiles, Tab<T> tg, Bat bt) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (rhs_skipped(bt)) return;
  A = wb(A, bt);
  A1 = wb(A1, bt);
  B2 = wb(B2, bt);
  T* lds = reinterpret_cast<T*>(smem);
  using S = TileCfg<T, N, DCT2>;
  static_assert(S::R1 == TileCfg<T, N, DST2>::R1 && S::M == TileCfg<T, N, DST2>::M, "one gather for both kinds");
  constexpr int W = S::W, R1 = S::R1;
  const Tab<T> tb = tables_to_lds<T, N, DCT2>(smem, tg);
  C2<T> raw[PipeCfg<T, N, DCT2>::PER];
  int tile = blockIdx.x;
  if (tile < ntiles) fetch_xy<T, N, DCT2>(A, tile_addr<W, N>(1, tile), raw);
  for (; tile < ntiles; tile += gridDim.x) {
    const TileAddr a = tile_addr<W, N>(1, tile);
    __syncthreads();  // the previous tile's outputs have been read from LDS
    stage_xy<T, N, DCT2>(lds, raw);
    __syncthreads();
    if (tile + (int)gridDim.x < ntiles) fetch_xy<T, N, DCT2>(A, tile_addr<W, N>(1, tile + gridDim.x), raw);
    const LdsSrc<T, N> src{lds};
    C2<T> zc[S::PT1][R1], zs[S::PT1][R1];
    fft_gather<T, N, DCT2>([&](int j, int n) { return pre_sample<T, N, DCT2>(src, tb, j, n); }, zc);
#pragma unroll
    for (int u = 0; u < S::PT1; ++u)
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) {
        const bool odd = S::M * n1 >= N / 2;  // as in ypair_fwd_body
        zs[u][n1] = odd ? C2<T>{-zc[u][n1].x, -zc[u][n1].y} : zc[u][n1];
      }
    fft_core_from<T, N, DST2>(lds, zs, tb);
    store_xy_outputs<T, N, DST2>(lds, tb, A1 + a.base, a.nstride);
    fft_core_from<T, N, DCT2>(lds, zc, tb);
    store_xy_outputs<T, N, DCT2>(lds, tb, B2 + a.base, a.nstride);
  }
}

// Persistent, pipelined form of the inverse y pair (as k_pass_pipe): per tile, the staged A1
// rows are transformed while the B2 rows of the same tile arrive in registers, and the staged
// B2 rows while the A1 rows of the block's next tile arrive.  The two inverse kinds share their
// tables (twiddles, mk, 1/s_k), which live in LDS.
template <typename T, int N>
__global__ __launch_bounds__(tile_nt_max<N>()) void k_ypair_inv_pipe(const T* __restrict__ A1, const T* __restrict__ B2,
                                                       T* __restrict__ A, int ntiles, Tab<T> tg, Bat bt) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (rhs_skipped(bt)) return;
  A1 = wb(A1, bt);
  B2 = wb(B2, bt);
  A = wb(A, bt);
  T* lds = reinterpret_cast<T*>(smem);
  using O = OutItems<T, N, DST3>;
  constexpr int W = TileCfg<T, N, DST3>::W;
  static_assert(PipeCfg<T, N, DST3>::PER == PipeCfg<T, N, DCT3>::PER, "one prefetch buffer for both kinds");
  const Tab<T> tb = tables_to_lds<T, N, DST3>(smem, tg);
  C2<T> raw[PipeCfg<T, N, DST3>::PER];
  int tile = blockIdx.x;
  if (tile < ntiles) fetch_xy<T, N, DST3>(A1, tile_addr<W, N>(1, tile), raw);
  for (; tile < ntiles; tile += gridDim.x) {
    const TileAddr a = tile_addr<W, N>(1, tile);
    __syncthreads();  // the previous tile's outputs have been read from LDS
    stage_xy<T, N, DST3>(lds, raw);
    __syncthreads();
    fetch_xy<T, N, DCT3>(B2, a, raw);
    fft_tile<T, N, DST3>(lds, LdsSrc<T, N>{lds}, tb);
    C2<T> acc[O::PER_XY];
#pragma unroll
    for (int u = 0; u < O::PER_XY; ++u) {
      int j, k;
      if (O::xy(u, j, k)) post_pair<T, N, DST3>(lds, tb, j, k, acc[u].x, acc[u].y);
    }
    __syncthreads();
    stage_xy<T, N, DCT3>(lds, raw);
    __syncthreads();
    if (tile + (int)gridDim.x < ntiles) fetch_xy<T, N, DST3>(A1, tile_addr<W, N>(1, tile + gridDim.x), raw);
    fft_tile<T, N, DCT3>(lds, LdsSrc<T, N>{lds}, tb);
    C2<T>* o = reinterpret_cast<C2<T>*>(A + a.base);
    const long ns = a.nstride / 2;
#pragma unroll
    for (int u = 0; u < O::PER_XY; ++u) {
      int j, k;
      if (O::xy(u, j, k)) {
        C2<T> v;
        post_pair<T, N, DCT3>(lds, tb, j, k, v.x, v.y);
        v.x += acc[u].x;
        v.y += acc[u].y;
        o[k * ns + j] = v;
      }
    }
  }
}

// CG coefficients after the matvec of iteration k, one block.  rpart: partial sums of r_k.r_k
// (nr blocks); zpart: partial sums (d.q, q, d, q.q) of q = S d_k (nz blocks).  With q' = q - mean q
// (Stokes) or q: alpha = r.r / d.q', and, by the conjugacy of d_k and d_{k-1},
// |r_{k+1}|^2 = alpha^2 q'.q' - r_k.r_k, so beta = |r_{k+1}|^2 / r_k.r_k is known before r_{k+1}
// is formed (the next forward z pass forms it together with x and d).
// scal: [0] |r_{k+1}|^2 (recurrence), [1] alpha, [2] beta, [3] mean q, [7] r_k.r_k
constexpr int CG_NT = 1024;  // threads of the coefficient kernel (its loads are latency-bound)
// hslot (may be null): pinned host memory, 8 doubles per right-hand side, that receives
// scal[0] and scal[7] of this iteration (the stop test reads them there, with no copy between
// the iteration's kernels and the next one)
__global__ __launch_bounds__(CG_NT) void k_cg_coef(const double* __restrict__ rpart, int nr,
                                                const double* __restrict__ zpart, int nz, double* __restrict__ scal,
                                                int stokes, int64_t M, Bat bt, double* __restrict__ hslot) {
  __shared__ double red[CG_NT / 64];
  if (rhs_skipped(bt)) return;
  rpart = wb(rpart, bt);
  zpart = wb(zpart, bt);
  scal = wb(scal, bt);
  double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll 2
  for (int i = threadIdx.x; i < nr; i += CG_NT) acc[0] += rpart[i];
  const double4* z4 = reinterpret_cast<const double4*>(zpart);
#pragma unroll 4
  for (int i = threadIdx.x; i < nz; i += CG_NT) {
    const double4 v = z4[i];
    acc[1] += v.x;
    acc[2] += v.y;
    acc[3] += v.z;
    acc[4] += v.w;
  }
  double tot[5];
  for (int c = 0; c < 5; ++c) tot[c] = block_sum(acc[c], red);
  if (threadIdx.x == 0) {
    const double rr = tot[0];
    const double mq = stokes ? tot[2] / (double)M : 0.0;
    const double dq = tot[1] - mq * tot[3];
    const double qq = tot[4] - (stokes ? mq * mq * (double)M : 0.0);
    const double alpha = (dq != 0.0) ? rr / dq : 0.0;
    double rn = alpha * alpha * qq - rr;
    // a non-positive estimate (cancellation near convergence, or lost conjugacy) restarts the
    // directions with beta = 0; the host never stops the solve on this estimate alone
    if (!(rn > 0.0)) rn = (rn == rn) ? 0.0 : rn;
    scal[0] = rn;
    scal[1] = alpha;
    scal[2] = (rr > 0.0) ? rn / rr : 0.0;
    scal[3] = mq;
    scal[7] = rr;
    if (hslot) {
      double* h = hslot + 8 * (int)blockIdx.z;
      h[0] = rn;
      h[7] = rr;
      __threadfence_system();  // visible to the host once the kernel has completed
    }
  }
}

// x += scal[idx] d
template <typename T>
__global__ __launch_bounds__(EW_NT) void k_axpy_scal(int64_t M, T* __restrict__ x, const T* __restrict__ d,
                                                  const double* __restrict__ scal, int idx, Bat bt) {
  if (rhs_skipped(bt)) return;
  x = wb(x, bt);
  d = wb(d, bt);
  scal = wb(scal, bt);
  const T a = T(scal[idx]);
  for (int64_t i = (int64_t)blockIdx.x * EW_NT + threadIdx.x; i < M; i += (int64_t)gridDim.x * EW_NT)
    x[i] += a * d[i];
}

template <typename T>
__global__ __launch_bounds__(EW_NT) void k_dot_partials(int64_t M, const T* __restrict__ a, const T* __restrict__ b,
                                                     double* __restrict__ partials) {
  __shared__ double red[EW_NT / 64];
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * EW_NT + threadIdx.x; i < M; i += (int64_t)gridDim.x * EW_NT)
    s += (double)a[i] * (double)b[i];
  double t = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

template <typename T>
__global__ __launch_bounds__(EW_NT) void k_sum_partials(int64_t M, const T* __restrict__ a, double* __restrict__ partials,
                                                     Bat bt) {
  __shared__ double red[EW_NT / 64];
  if (rhs_skipped(bt)) return;
  a = wb(a, bt);
  partials = wb(partials, bt);
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * EW_NT + threadIdx.x; i < M; i += (int64_t)gridDim.x * EW_NT) s += (double)a[i];
  double t = block_sum(s, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// hdst (may be null): pinned host memory that also receives the residual norm scal[5] of the
// R_RESNORM / R_RESNORM0 ops, one double per right-hand side (read by the host after a
// synchronisation, with no copy operation on the stream)
__global__ __launch_bounds__(EW_NT) void k_reduce(const double* __restrict__ partials, int nparts, int nper,
                                               double* __restrict__ scal, int op, int stokes, int64_t M,
                                               double* __restrict__ out, Bat bt, double* __restrict__ hdst) {
  __shared__ double red[EW_NT / 64];
  if (rhs_skipped(bt)) return;
  partials = wb(partials, bt);
  scal = wb(scal, bt);
  out = wb(out, bt);
  double acc[4] = {0, 0, 0, 0};
  for (int i = threadIdx.x; i < nparts; i += EW_NT)
    for (int c = 0; c < nper; ++c) acc[c] += partials[(int64_t)i * nper + c];
  double tot[4];
  for (int c = 0; c < 4; ++c) tot[c] = block_sum(c < nper ? acc[c] : 0.0, red);
  if (threadIdx.x == 0) {
    if (op == R_RESNORM || op == R_RESNORM0) {
      // |r_u|^2 + |r_p - mean r_p|^2 (Stokes: the pressure equation is taken modulo constants);
      // R_RESNORM0 also keeps the mean of the pressure part in scal[6]
      scal[5] = tot[0] + tot[2] - (stokes ? tot[1] * tot[1] / (double)M : 0.0);
      if (op == R_RESNORM0) scal[6] = tot[1] / (double)M;
      if (hdst) {
        hdst[blockIdx.z] = scal[5];
        __threadfence_system();
      }
    } else {
      const double v = (op == R_SUM1) ? tot[1] : tot[0];
      if (out)
        *out = v;
      else
        scal[5] = v;
    }
  }
}

template <typename T>
__global__ void k_add_scalar(int64_t M, T* a, const double* scal, int idx, double factor, Bat bt) {
  if (rhs_skipped(bt)) return;
  a = wb(a, bt);
  scal = wb(scal, bt);
  const T v = T(scal[idx] * factor);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x)
    a[i] += v;
}


// ---------------------------------------------------------------------------------------
// elementwise
// ---------------------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(int64_t n, T* a, T v, Bat bt) {
  if (rhs_skipped(bt)) return;
  a = wb(a, bt);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}
template <typename T>
__global__ void k_axpby(int64_t n, T* y, double a, const T* x, double b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = T(a * (double)x[i] + b * (double)y[i]);
}

// ---------------------------------------------------------------------------------------
// full-system MAC residual (float64, internal layout)
// ---------------------------------------------------------------------------------------


// ---------------------------------------------------------------------------------------
// mixed-precision refinement (float64 residual of the full MAC system, float32 correction)
// ---------------------------------------------------------------------------------------
// r32 = (float) F (four fields, unshifted: the first inner solve projects the mean of its
// pressure right-hand side itself, and F_p is not small against its mean); per-block partial
// sums of F_u.F_u, sum F_p, F_p.F_p
__global__ __launch_bounds__(EW_NT) void k_refine_prep(int64_t M, const double* __restrict__ F,
                                                    float* __restrict__ r32, double* __restrict__ partials,
                                                    Bat bt) {
  __shared__ double red[EW_NT / 64];
  if (rhs_skipped(bt)) return;
  F = wb(F, bt);
  r32 = wb(r32, bt);
  partials = wb(partials, bt);
  double su = 0, sp = 0, spp = 0;
  // the four fields as one flat array, four values per thread (M is a multiple of 4): 32-byte
  // loads, 16-byte stores, one stream at a time instead of four 2^k-apart streams
  const int64_t G = M;  // groups of four over 4M values
  for (int64_t g = (int64_t)blockIdx.x * EW_NT + threadIdx.x; g < G; g += (int64_t)gridDim.x * EW_NT) {
    const int64_t i = g << 2;
    const double4 v = *reinterpret_cast<const double4*>(F + i);
    *reinterpret_cast<float4*>(r32 + i) = float4{(float)v.x, (float)v.y, (float)v.z, (float)v.w};
    const double q = v.x * v.x + v.y * v.y + v.z * v.z + v.w * v.w;
    if (i < 3 * M) {
      su += q;
    } else {
      sp += (v.x + v.y) + (v.z + v.w);
      spp += q;
    }
  }
  const double t0 = block_sum(su, red), t1 = block_sum(sp, red), t2 = block_sum(spp, red);
  if (threadIdx.x == 0) {
    partials[3 * blockIdx.x] = t0;
    partials[3 * blockIdx.x + 1] = t1;
    partials[3 * blockIdx.x + 2] = t2;
  }
}

// One refinement update and the new residual, in one pass over the cells (internal layout,
// z fastest): u' = u + x32_u, p' = p + x32_p (u = p = 0 in the first round), then
//   r_u = F_u - (-mu lap_h u' + G p'),   r_p = F_p - (D u' + c p')
// in float64 (face 0 and face N of each u_m are the box faces, zero; tangential ghosts by
// reflection), written as float32 for the next inner solve, with per-block partial sums of
// r_u.r_u and of the shifted r_p and r_p.r_p.  The pressure part is shifted by -(*shift)
// (Stokes: the mean of F_p, which the residual keeps; left in, the float32 inner solve would
// have to cancel an O(|F|) constant against an O(1e-5 |F|) residual and stagnates).  Neighbour values of u' are formed on the fly, so u', p' go to
// buffers other than u, p.
// WRITE = false: the residual norms only (the partial sums); nothing else is written, for a
// first round whose result is then read from x32 itself when it meets the tolerance
template <bool FIRST, bool WRITE>
__global__ __launch_bounds__(EW_NT) void k_refine_residual(int N, double h, double mu, double cc,
                                                        const double* __restrict__ u, const double* __restrict__ p,
                                                        const float* __restrict__ x32, const double* __restrict__ F,
                                                        const double* __restrict__ shift, double* __restrict__ un,
                                                        double* __restrict__ pn, float* __restrict__ r32,
                                                        double* __restrict__ partials, Bat bt,
                                                        const uint8_t* __restrict__ fmask) {
  __shared__ double red[EW_NT / 64];
  if (rhs_skipped(bt)) return;
  u = wb(u, bt);
  p = wb(p, bt);
  x32 = wb(x32, bt);
  F = wb(F, bt);
  shift = wb(shift, bt);
  un = wb(un, bt);
  pn = wb(pn, bt);
  r32 = wb(r32, bt);
  partials = wb(partials, bt);
  const double sh = shift ? *shift : 0.0;
  // N is a power of two and N^3 < 2^31 (N <= 512): 32-bit indices, shifts and masks
  const int lg = __builtin_ctz(N), mask = N - 1;
  const int M = N << (2 * lg);
  const double ih2 = 1.0 / (h * h), ih = 1.0 / h;
  const int st[3] = {N * N, N, 1};
  auto U = [&](int m, int j) -> double {
    const double v = (double)x32[(int64_t)m * M + j];
    return FIRST ? v : u[(int64_t)m * M + j] + v;
  };
  auto P = [&](int j) -> double {
    const double v = (double)x32[(int64_t)3 * M + j];
    return FIRST ? v : p[j] + v;
  };
  // XCD-aware chunking: the hardware deals workgroups round-robin over the 8 XCDs, so block b
  // takes logical chunk (b % 8) * (nb / 8) + b / 8 and each XCD sweeps one contiguous slab of
  // x-planes; the x, y and z neighbours of a point are then read by blocks of the same XCD
  // (same L2) at about the same time.  gridDim.x is a multiple of 8.
  const int nb = gridDim.x;
  const int L = (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
  const int chunk = (M + nb - 1) / nb;
  const int i1 = (L + 1) * chunk < M ? (L + 1) * chunk : M;
  // fmask (may be null): per z-pencil bits of the components of F that can be nonzero; a
  // wavefront covers 64 cells of one pencil when N >= 64 and the chunks are 64-aligned, so its
  // flags are read once per wavefront and the loads of zero F entries are skipped as a whole
  const bool wave_pencil = N >= 64 && chunk % 64 == 0;
  double su = 0, sp = 0, spp = 0;
  for (int i = L * chunk + threadIdx.x; i < i1; i += EW_NT) {
    const int id[3] = {i >> (2 * lg), (i >> lg) & mask, i & mask};
    unsigned fm = 0xFu;
    if (fmask) fm = wave_pencil ? fmask[__builtin_amdgcn_readfirstlane(i >> lg)] : fmask[i >> lg];
    const double pc = P(i);
    double div = 0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      // every neighbour is loaded unconditionally (clamped to the point itself) and replaced
      // by its boundary value afterwards, so all loads of a point are in flight together
      const double cu = U(m, i);
      const double c = (id[m] == 0) ? 0.0 : cu;  // face 0 is the box face
      double lap = 0, hi_m = 0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const bool lo_ok = (d == m) ? id[d] > 1 : id[d] > 0;
        const bool hi_ok = id[d] + 1 < N;
        const double vlo = U(m, lo_ok ? i - st[d] : i);
        const double vhi = U(m, hi_ok ? i + st[d] : i);
        // face a-1 / face N: zero (box faces); tangential ghosts: reflection -c
        const double lo = lo_ok ? vlo : (d == m ? 0.0 : -c);
        const double hi = hi_ok ? vhi : (d == m ? 0.0 : -c);
        if (d == m) hi_m = hi;
        lap += (lo - 2.0 * c + hi) * ih2;
      }
      div += (hi_m - c) * ih;
      const double gp = (pc - P(id[m] > 0 ? i - st[m] : i)) * ih;  // cells a-1, a
      const double fv = ((fm >> m) & 1u) ? F[(int64_t)m * M + i] : 0.0;
      const double r = (id[m] > 0) ? fv - (-mu * lap + gp) : 0.0;
      if constexpr (WRITE) {
        un[(int64_t)m * M + i] = c;
        r32[(int64_t)m * M + i] = (float)r;
      }
      su += r * r;
    }
    const double rp = (((fm >> 3) & 1u) ? F[(int64_t)3 * M + i] : 0.0) - (div + cc * pc) - sh;
    if constexpr (WRITE) {
      pn[i] = pc;
      r32[(int64_t)3 * M + i] = (float)rp;
    }
    sp += rp;
    spp += rp * rp;
  }
  const double t0 = block_sum(su, red), t1 = block_sum(sp, red), t2 = block_sum(spp, red);
  if (threadIdx.x == 0) {
    partials[3 * blockIdx.x] = t0;
    partials[3 * blockIdx.x + 1] = t1;
    partials[3 * blockIdx.x + 2] = t2;
  }
}

// ---------------------------------------------------------------------------------------
// surface stages (float64)
// ---------------------------------------------------------------------------------------
// Eight lanes per crossing t (lane q < 6 owns fit quantity q: value, two first and three second
// tangential derivatives, for the three components), so that the fit weights of one
// neighbour entry (6 doubles) are read as one contiguous segment; the 5 jumps of the crossing
// are then reduced over the lanes of the group.  jmap is component-major on the device,
// jmap[(r * 18 + c) * T + t]; fit values are kept only for the control points
// (fitvals[18 cp + c]), which the interpolation jump needs.
constexpr int FJ_LANES = 8;
// work buffer of right-hand side r (batched launches serve several per block)
template <typename P>
__device__ __forceinline__ P wbr(P p, const Bat& b, int r) {
  return reinterpret_cast<P>(reinterpret_cast<uintptr_t>(p) + (uint64_t)r * (uint64_t)b.A);
}
__global__ __launch_bounds__(256) void k_fit_jump(int64_t T, const int64_t* __restrict__ nb_ptr,
                                                 const int32_t* __restrict__ nb_idx, const double* __restrict__ fitw,
                                                 const double* __restrict__ jmap, const double* __restrict__ jfmap,
                                                 const double* __restrict__ Fj, const double* __restrict__ phi,
                                                 const int64_t* __restrict__ cp_of, double* __restrict__ jumps,
                                                 double* __restrict__ fitvals, Bat bt) {
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FJ_LANES;
  const int q = threadIdx.x % FJ_LANES;
  const bool live = t < T;  // all lanes stay for the shuffles
  // right-hand sides r0 .. r0 + nr - 1 of this group (nr is uniform over the block)
  const int r0 = FJ_RHS * (int)blockIdx.z;
  const int nr = min(FJ_RHS, bt.nb - r0);
  double fv[FJ_RHS][3];
#pragma unroll
  for (int rr = 0; rr < FJ_RHS; ++rr) fv[rr][0] = fv[rr][1] = fv[rr][2] = 0.0;
  if (live && q < 6) {
    for (int64_t e = nb_ptr[t]; e < nb_ptr[t + 1]; ++e) {
      const int64_t cp = nb_idx[e];
      const double w = fitw[6 * e + q];
#pragma unroll
      for (int rr = 0; rr < FJ_RHS; ++rr)
        if (rr < nr) {
          const double* ph = phi + (int64_t)(r0 + rr) * bt.U;
          fv[rr][0] += w * ph[3 * cp];
          fv[rr][1] += w * ph[3 * cp + 1];
          fv[rr][2] += w * ph[3 * cp + 2];
        }
    }
    const int64_t cp = cp_of[t];
    if (cp >= 0)
#pragma unroll
      for (int rr = 0; rr < FJ_RHS; ++rr)
        if (rr < nr)
          for (int i = 0; i < 3; ++i) wbr(fitvals, bt, r0 + rr)[18 * cp + 3 * q + i] = fv[rr][i];
  }
  double part[FJ_RHS][5];
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    double jm[3] = {0.0, 0.0, 0.0};
    if (live && q < 6)
      for (int i = 0; i < 3; ++i) jm[i] = jmap[(int64_t)(r * 18 + 3 * q + i) * T + t];
#pragma unroll
    for (int rr = 0; rr < FJ_RHS; ++rr) {
      part[rr][r] = 0.0;
      if (rr < nr) {
        double s = jm[0] * fv[rr][0] + jm[1] * fv[rr][1] + jm[2] * fv[rr][2];
#pragma unroll
        for (int o = 1; o < FJ_LANES; o <<= 1) s += __shfl_xor(s, o, FJ_LANES);
        part[rr][r] = s;
      }
    }
  }
  if (live && q < 5) {
#pragma unroll
    for (int rr = 0; rr < FJ_RHS; ++rr)
      if (rr < nr) {
        double s = part[rr][0];
#pragma unroll
        for (int r = 1; r < 5; ++r)
          if (q == r) s = part[rr][r];
        if (Fj) {
          const double* Fr = jfmap + (t * 5 + q) * 3;
          s += Fr[0] * Fj[3 * t] + Fr[1] * Fj[3 * t + 1] + Fr[2] * Fj[3 * t + 2];
        }
        wbr(jumps, bt, r0 + rr)[5 * t + q] = s;
      }
  }
}

__global__ void k_interp_jump(int64_t n, const int64_t* __restrict__ cp_target, const double* __restrict__ fitvals,
                              const double* __restrict__ emap, const double* __restrict__ efmap,
                              const double* __restrict__ Fj, double* __restrict__ ejump, Bat bt) {
  if (rhs_skipped(bt)) return;
  fitvals = wb(fitvals, bt);
  ejump = wb(ejump, bt);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 3 * n) return;
  const int64_t c = r / 3;
  const int64_t t = cp_target[c];
  double s = 0;
  for (int q = 0; q < 18; ++q) s += emap[18 * r + q] * fitvals[18 * c + q];
  if (Fj)
    for (int i = 0; i < 3; ++i) s += efmap[3 * r + i] * Fj[3 * t + i];
  ejump[r] = s;
}

// Correction of every irregular node, assigned into F (every irregular node appears once, its
// equation's arms being grouped).  With r32 != nullptr the float32 copy is assigned as well and
// the block writes the partial sums (F_u.F_u, sum F_p, F_p.F_p) over its nodes to partials[3b..]:
// when F is zero elsewhere, these are the refinement's start values without a dense pass.
__global__ __launch_bounds__(EW_NT) void k_correct(int64_t nirr, const int64_t* __restrict__ irr_node,
                                                const int64_t* __restrict__ irr_ptr,
                                                const int32_t* __restrict__ arm_t, const int8_t* __restrict__ arm_o,
                                                const double* __restrict__ arm_a, const double* __restrict__ jumps,
                                                double* __restrict__ F, float* __restrict__ r32, int64_t M,
                                                double* __restrict__ partials, Bat bt) {
  __shared__ double red[EW_NT / 64];
  if (rhs_skipped(bt)) return;
  jumps = wb(jumps, bt);
  F = wb(F, bt);
  r32 = wb(r32, bt);
  partials = wb(partials, bt);
  double su = 0, sp = 0, spp = 0;
  for (int64_t r = (int64_t)blockIdx.x * EW_NT + threadIdx.x; r < nirr; r += (int64_t)gridDim.x * EW_NT) {
    double v = 0;
    for (int64_t q = irr_ptr[r]; q < irr_ptr[r + 1]; ++q) {
      const double* J = jumps + 5 * (int64_t)arm_t[q] + arm_o[q];
      const double* a = arm_a + 3 * q;
      v += a[0] * J[0] + a[1] * J[1];
      if (arm_o[q] == 0) v += a[2] * J[2];
    }
    const int64_t node = irr_node[r];
    F[node] = v;
    if (r32) {
      r32[node] = (float)v;
      if (node < 3 * M) {
        su += v * v;
      } else {
        sp += v;
        spp += v * v;
      }
    }
  }
  if (r32) {
    const double t0 = block_sum(su, red), t1 = block_sum(sp, red), t2 = block_sum(spp, red);
    if (threadIdx.x == 0) {
      partials[3 * blockIdx.x] = t0;
      partials[3 * blockIdx.x + 1] = t1;
      partials[3 * blockIdx.x + 2] = t2;
    }
  }
}

__global__ void k_interp(int64_t n, const int64_t* __restrict__ idx, const double* __restrict__ w,
                         const double* __restrict__ u, const double* __restrict__ ejump, double* __restrict__ out,
                         Bat bt) {
  if (rhs_skipped(bt)) return;
  u = wb(u, bt);
  ejump = wb(ejump, bt);
  out = ub(out, bt);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 3 * n) return;
  double s = ejump[r];
#pragma unroll
  for (int q = 0; q < 10; ++q) s += w[10 * r + q] * u[idx[10 * r + q]];
  out[r] = s;
}

// The same from the float32 first-round solution x32 of the mixed solve (velocity components
// in the layout of u): the float64 iterate of that round is x32 itself with face 0 of each
// component (the box face) at zero, read here without being stored.
__global__ void k_interp_x32(int64_t n, const int64_t* __restrict__ idx, const double* __restrict__ w,
                             const float* __restrict__ x32, int lg, const double* __restrict__ ejump,
                             double* __restrict__ out, Bat bt) {
  if (rhs_skipped(bt)) return;
  x32 = wb(x32, bt);
  ejump = wb(ejump, bt);
  out = ub(out, bt);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 3 * n) return;
  const int64_t M = (int64_t)1 << (3 * lg), mask = ((int64_t)1 << lg) - 1;
  double s = ejump[r];
#pragma unroll
  for (int q = 0; q < 10; ++q) {
    const int64_t g = idx[10 * r + q];
    const int m = (int)(g >> (3 * lg));
    const int64_t i = g & (M - 1);
    const int64_t face = (i >> (lg * (2 - m))) & mask;  // index along axis m
    const double v = face == 0 ? 0.0 : (double)x32[g];
    s += w[10 * r + q] * v;
  }
  out[r] = s;
}

// average trace form (control point c, component m, r = 3c + m):
//   out[r] += a[r] (phi[r] - sum_e sw[e] phi[3 idx[e] + m]),  a = 1/2 - exterior weight fraction
__global__ void k_stab(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx,
                       const double* __restrict__ sw, const double* __restrict__ a, const double* __restrict__ phi,
                       double* __restrict__ out, Bat bt) {
  if (rhs_skipped(bt)) return;
  phi = ub(phi, bt);
  out = ub(out, bt);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 3 * n) return;
  const int64_t c = r / 3;
  const int m = (int)(r - 3 * c);
  double s = 0;
  for (int64_t e = ptr[c]; e < ptr[c + 1]; ++e) s += sw[e] * phi[3 * (int64_t)idx[e] + m];
  out[r] += a[r] * (phi[r] - s);
}

// its transpose, gathered over the transposed CSR (rows ascending):
//   out[r] += a[r] w[r] - sum_e swT[e] a[3 row[e] + m] w[3 row[e] + m]
__global__ void k_stab_T(int64_t n, const int64_t* __restrict__ ptr, const int32_t* __restrict__ row,
                         const double* __restrict__ sw, const double* __restrict__ a, const double* __restrict__ w,
                         double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 3 * n) return;
  const int64_t j = r / 3;
  const int m = (int)(r - 3 * j);
  double s = a[r] * w[r];
  for (int64_t e = ptr[j]; e < ptr[j + 1]; ++e) {
    const int64_t q = 3 * (int64_t)row[e] + m;
    s -= sw[e] * a[q] * w[q];
  }
  out[r] += s;
}

__global__ void k_interp8(int64_t m, const int64_t* __restrict__ idx, const double* __restrict__ w,
                          const double* __restrict__ u, double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 3 * m) return;
  double s = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += w[8 * r + q] * u[idx[8 * r + q]];
  out[r] = s;
}

__global__ void k_interp_T(int64_t nnode, const int64_t* __restrict__ ptr, const int64_t* __restrict__ node,
                           const int32_t* __restrict__ row, const double* __restrict__ w,
                           const double* __restrict__ wbar, double* __restrict__ ubar) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnode) return;
  double s = 0;
  for (int64_t e = ptr[k]; e < ptr[k + 1]; ++e) s += w[e] * wbar[row[e]];
  ubar[node[k]] = s;
}

__global__ void k_correct_T(int64_t T, const int64_t* __restrict__ ptr, const int64_t* __restrict__ node,
                            const int8_t* __restrict__ slot, const double* __restrict__ a,
                            const double* __restrict__ Fbar, double* __restrict__ jbar) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  double s[5] = {0, 0, 0, 0, 0};
  for (int64_t e = ptr[t]; e < ptr[t + 1]; ++e) s[slot[e]] += a[e] * Fbar[node[e]];
  for (int q = 0; q < 5; ++q) jbar[5 * t + q] = s[q];
}

__global__ void k_jump_T(int64_t T, const int64_t* __restrict__ cp_of, const double* __restrict__ jmap,
                         const double* __restrict__ emap, const double* __restrict__ jbar,
                         const double* __restrict__ wbar, double* __restrict__ fitbar) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const int64_t cp = cp_of[t];
  for (int c = 0; c < 18; ++c) {
    double s = 0;
    for (int r = 0; r < 5; ++r) s += jmap[(r * 18 + c) * T + t] * jbar[5 * t + r];
    if (cp >= 0 && wbar)
      for (int m = 0; m < 3; ++m) s += emap[(cp * 3 + m) * 18 + c] * wbar[3 * cp + m];
    fitbar[18 * t + c] = s;
  }
}

__global__ void k_fit_T(int64_t n, const int64_t* __restrict__ ptr, const int64_t* __restrict__ entry,
                        const int32_t* __restrict__ target, const double* __restrict__ fitw,
                        const double* __restrict__ fitbar, double* __restrict__ phibar) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double s[3] = {0, 0, 0};
  for (int64_t q = ptr[c]; q < ptr[c + 1]; ++q) {
    const int64_t e = entry[q];
    const double* fb = fitbar + 18 * (int64_t)target[q];
    for (int k = 0; k < 6; ++k) {
      const double w = fitw[6 * e + k];
      s[0] += w * fb[3 * k];
      s[1] += w * fb[3 * k + 1];
      s[2] += w * fb[3 * k + 2];
    }
  }
  phibar[3 * c] = s[0];
  phibar[3 * c + 1] = s[1];
  phibar[3 * c + 2] = s[2];
}

__global__ void k_export_u(int N, const double* __restrict__ ui, double* __restrict__ ue) {
  const int64_t M = (int64_t)N * N * N;
  const int64_t Me = (int64_t)(N + 1) * N * N;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < 3 * Me; g += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(g / Me);
    const int64_t l = g - m * Me;
    int sh[3] = {N, N, N};
    sh[m] = N + 1;
    const int k = (int)(l % sh[2]), j = (int)((l / sh[2]) % sh[1]), i = (int)(l / ((int64_t)sh[2] * sh[1]));
    const int id[3] = {i, j, k};
    double v = 0.0;
    if (id[m] < N) v = ui[m * M + ((int64_t)i * N + j) * N + k];
    ue[g] = v;
  }
}

__global__ void k_import_u(int N, const double* __restrict__ ue, double* __restrict__ ui) {
  const int64_t M = (int64_t)N * N * N;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < 3 * M; g += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(g / M);
    const int64_t l = g - m * M;
    const int k = (int)(l % N), j = (int)((l / N) % N), i = (int)(l / ((int64_t)N * N));
    int sh[3] = {N, N, N};
    sh[m] = N + 1;
    const int64_t Me = (int64_t)(N + 1) * N * N;
    const int id[3] = {i, j, k};
    ui[g] = (id[m] == 0) ? 0.0 : ue[m * Me + ((int64_t)i * sh[1] + j) * sh[2] + k];
  }
}

__global__ void k_scatter_add(int64_t n, const int64_t* __restrict__ idx, const double* __restrict__ v,
                              double* __restrict__ F) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) F[idx[r]] += v[r];
}

template <typename Ti, typename To>
__global__ void k_convert(int64_t n, const Ti* __restrict__ in, To* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (To)in[i];
}

// flag: pinned host memory (its device address), read by the host after a synchronisation;
// a non-finite entry stores the call's tag there, so a store left over from an earlier check
// can never be taken for this one
__global__ void k_check_finite(int64_t n, const double* __restrict__ a, int* __restrict__ flag, int tag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(a[i])) {
      *flag = tag;  // benign race: every writer stores the same value
      __threadfence_system();
    }
}

// ---------------------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------------------
static inline int ew_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

// kernels whose tile needs more than the default 64 KiB of LDS opt in to the larger limit
template <typename K>
static void ensure_lds(K kernel, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

#define KFBI_DISPATCH_N(N, MACRO) \
  switch (N) {                    \
    case 16: MACRO(16); break;    \
    case 32: MACRO(32); break;    \
    case 64: MACRO(64); break;    \
    case 128: MACRO(128); break;  \
    case 256: MACRO(256); break;  \
    case 512: MACRO(512); break;  \
    default: return hipErrorInvalidValue; \
  }

template <typename T, int N, int KIND, bool ACC>
static hipError_t pass_n(int axis, const T* in, T* out, const Tab<T>& tb, hipStream_t s, const Bat& bt,
                         const uint8_t* pmask, const uint8_t* xmask, int mbit) {
  using S = TileCfg<T, N, KIND>;
  const size_t lds = TabStage<T, N, KIND>::BYTES;  // (S::BYTES where the table stage is off)
  const int blocks = N * N / S::W;
  // the inverse kinds read two samples per FFT input, which the staged tile serves from LDS;
  // for the forward kinds the direct gather measured faster
  if constexpr (PipeCfg<T, N, KIND>::BYTES <= 163840 && !ACC && (KIND == DCT3 || KIND == DST3)) {
    if (axis != 2) {
      using P = PipeCfg<T, N, KIND>;
      ensure_lds(k_pass_pipe<T, N, KIND>, P::BYTES);
      static std::atomic<int> per_cu{0};
      const int pb = persistent_blocks(k_pass_pipe<T, N, KIND>, S::NT, P::BYTES, blocks, per_cu);
      hipLaunchKernelGGL((k_pass_pipe<T, N, KIND>), dim3(pb, 1, bt.nb), dim3(S::NT), P::BYTES, s, in, out, axis, blocks,
                         tb, bt);
      return hipGetLastError();
    }
  }
  ensure_lds(k_pass<T, N, KIND, ACC>, lds);
  hipLaunchKernelGGL((k_pass<T, N, KIND, ACC>), dim3(blocks, 1, bt.nb), dim3(S::NT), lds, s, in, out, axis, tb, bt,
                     pmask, xmask, mbit);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t pass_kind(int kind, int axis, const T* in, T* out, bool acc, const Tab<T>& tb, hipStream_t s,
                            const Bat& bt, const uint8_t* pm, const uint8_t* xm, int mbit) {
#define KFBI_K(KD)                                                                                          \
  case KD:                                                                                                  \
    return acc ? pass_n<T, N, KD, true>(axis, in, out, tb, s, bt, pm, xm, mbit)                             \
               : pass_n<T, N, KD, false>(axis, in, out, tb, s, bt, pm, xm, mbit);
  switch (kind) {
    KFBI_K(DCT2)
    KFBI_K(DST2)
    KFBI_K(DCT3)
    KFBI_K(DST3)
    KFBI_K(DST1)
  }
#undef KFBI_K
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_pass(int N, int kind, int axis, const T* in, T* out, bool accumulate, const DevTables<T>& tb,
                       hipStream_t s, const Bat& bt, const uint8_t* pmask, const uint8_t* xmask, int mbit) {
  if (pmask && (!xmask || mbit < 0 || mbit > 7)) return hipErrorInvalidValue;
  const Tab<T> t = tab_of(tb);
#define KFBI_M(NN) return pass_kind<T, NN>(kind, axis, in, out, accumulate, t, s, bt, pmask, xmask, mbit)
  KFBI_DISPATCH_N(N, KFBI_M)
#undef KFBI_M
  return hipErrorInvalidValue;
}


template <typename T>
hipError_t launch_xmid(int N, T* A0, T* A1, T* A2, double mu, const DevTables<T>& tb, hipStream_t s, const Bat& bt) {
  const Tab<T> t = tab_of(tb);
#define KFBI_M(NN)                                                                                              \
  {                                                                                                             \
    using S = TileCfg<T, NN, DCT2>;                                                                             \
    const int blocks = NN * NN / S::W;                                                                          \
    const size_t lds = XmidLds<T, NN>::BYTES;                                                                   \
    ensure_lds(k_xmid<T, NN>, lds);                                                                             \
    hipLaunchKernelGGL((k_xmid<T, NN>), dim3(blocks, 3, bt.nb), dim3(S::NT), lds, s, A0, A1, A2, mu, t, bt);    \
  }
  KFBI_DISPATCH_N(N, KFBI_M)
#undef KFBI_M
  return hipGetLastError();
}

template <typename T>
hipError_t launch_zfwd_cg(int N, int mode, T* x, T* r, T* d, const T* q, T* A, T* B, const double* scal,
                          double* rpart, const DevTables<T>& tb, hipStream_t s, const Bat& bt) {
  const Tab<T> t = tab_of(tb);
#define KFBI_ZF(NN, MODE)                                                                                  \
  {                                                                                                        \
    using S = TileCfg<T, NN, DST2>;                                                                        \
    const int blocks = NN * NN / S::W;                                                                     \
    const size_t lds = TabStage<T, NN, DST2>::BYTES;                                                       \
    ensure_lds(k_zfwd_cg<T, NN, MODE>, lds);                                                               \
    hipLaunchKernelGGL((k_zfwd_cg<T, NN, MODE>), dim3(blocks, 1, bt.nb), dim3(S::NT), lds, s, x, r, d, q, A, B, \
                       scal, rpart, t, bt);                                                                \
  }
#define KFBI_M(NN)            \
  {                           \
    if (mode == ZF_FUSED)     \
      KFBI_ZF(NN, ZF_FUSED)   \
    else if (mode == ZF_FIRST) \
      KFBI_ZF(NN, ZF_FIRST)   \
    else if (mode == ZF_FINAL) \
      KFBI_ZF(NN, ZF_FINAL)   \
    else                      \
      KFBI_ZF(NN, ZF_PLAIN)   \
  }
  KFBI_DISPATCH_N(N, KFBI_M)
#undef KFBI_M
#undef KFBI_ZF
  return hipGetLastError();
}

int zfwd_blocks(int N, int elem_size) { return N * N / std::min(128 / elem_size, N); }
int zinv_blocks(int N, int elem_size) { return N * N / std::min(128 / elem_size, N); }

template <typename T>
hipError_t launch_zinv_cg(int N, const T* A, const T* B, T* q, const T* d, double c, double* partials,
                          const DevTables<T>& tb, hipStream_t s, const Bat& bt) {
  const Tab<T> t = tab_of(tb);
#define KFBI_M(NN)                                                                                         \
  {                                                                                                        \
    using S = TileCfg<T, NN, DCT3>;                                                                        \
    const int blocks = NN * NN / S::W;                                                                     \
    const size_t lds = TabStage<T, NN, DST3>::BYTES;                                                       \
    ensure_lds(k_zinv_cg<T, NN>, lds);                                                                     \
    hipLaunchKernelGGL((k_zinv_cg<T, NN>), dim3(blocks, 1, bt.nb), dim3(S::NT), lds, s, A, B, q, d, c,     \
                       partials, t, bt);                                                                   \
  }
  KFBI_DISPATCH_N(N, KFBI_M)
#undef KFBI_M
  return hipGetLastError();
}

template <typename T, int N, int KF, int KI, bool BS>
static hipError_t xfuse_n(int m, const T* in, T* fh, T* out, double mu, const DevTables<T>& tb, hipStream_t s,
                          const Bat& bt) {
  using SF = TileCfg<T, N, KF>;
  using SI = TileCfg<T, N, KI>;
  const size_t lds = XfuseLds<T, N, KF, KI>::BYTES;
  const int nt = SF::NT > SI::NT ? SF::NT : SI::NT;
  const int blocks = N * N / SF::W;
  ensure_lds(k_xfuse<T, N, KF, KI, BS>, lds);
  hipLaunchKernelGGL((k_xfuse<T, N, KF, KI, BS>), dim3(blocks, 1, bt.nb), dim3(nt), lds, s, in, fh, out, m, mu,
                     tab_of(tb), bt);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_xfuse(int N, int m, bool backsub, const T* in, T* fh, T* out, double mu, const DevTables<T>& tb,
                        hipStream_t s, const Bat& bt) {
  if (m < 0 || m > 2) return hipErrorInvalidValue;
#define KFBI_M(NN)                                                                            \
  if (backsub)                                                                                \
    return m == 0 ? xfuse_n<T, NN, DCT2, DST1, true>(m, in, fh, out, mu, tb, s, bt)           \
                  : xfuse_n<T, NN, DST2, DST3, true>(m, in, fh, out, mu, tb, s, bt);          \
  return m == 0 ? xfuse_n<T, NN, DST1, DCT3, false>(m, in, fh, out, mu, tb, s, bt)            \
                : xfuse_n<T, NN, DST2, DST3, false>(m, in, fh, out, mu, tb, s, bt);
  KFBI_DISPATCH_N(N, KFBI_M)
#undef KFBI_M
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_ypair(int N, bool inverse, const T* in0, const T* in1, T* out0, T* out1, const DevTables<T>& tb,
                        hipStream_t s, const Bat& bt) {
  const Tab<T> t = tab_of(tb);
#define KFBI_M(NN)                                                                                        \
  {                                                                                                       \
    using S = TileCfg<T, NN, DCT2>;                                                                       \
    const int blocks = NN * NN / S::W;                                                                    \
    const size_t lds = S::BYTES;                                                                          \
    using P = PipeCfg<T, NN, DST3>;                                                                       \
    if (inverse && NN <= 512 && P::BYTES <= 163840) {                                                     \
      ensure_lds(k_ypair_inv_pipe<T, NN>, P::BYTES);                                                      \
      static std::atomic<int> per_cu{0};                                                                  \
      const int pb = persistent_blocks(k_ypair_inv_pipe<T, NN>, S::NT, P::BYTES, blocks, per_cu);         \
      hipLaunchKernelGGL((k_ypair_inv_pipe<T, NN>), dim3(pb, 1, bt.nb), dim3(S::NT), P::BYTES, s, in0, in1, out0, \
                         blocks, t, bt);                                                                  \
    } else if (inverse) {                                                                                 \
      ensure_lds(k_ypair_inv<T, NN>, lds);                                                                \
      hipLaunchKernelGGL((k_ypair_inv<T, NN>), dim3(blocks, 1, bt.nb), dim3(S::NT), lds, s, in0, in1, out0, t, bt); \
    } else if (sizeof(T) == 4 && NN <= 512 && PipeCfg<T, NN, DCT2>::BYTES <= 163840) { \
      using PF = PipeCfg<T, NN, DCT2>;                                                                    \
      ensure_lds(k_ypair_fwd_pipe<T, NN>, PF::BYTES);                                                     \
      static std::atomic<int> per_cu_f{0};                                                                \
      const int pb = persistent_blocks(k_ypair_fwd_pipe<T, NN>, S::NT, PF::BYTES, blocks, per_cu_f);      \
      hipLaunchKernelGGL((k_ypair_fwd_pipe<T, NN>), dim3(pb, 1, bt.nb), dim3(S::NT), PF::BYTES, s, in0, out0, out1, \
                         blocks, t, bt);                                                                  \
    } else {                                                                                              \
      const size_t ldsf = TabStage<T, NN, DCT2>::BYTES;                                                   \
      ensure_lds(k_ypair_fwd<T, NN>, ldsf);                                                               \
      hipLaunchKernelGGL((k_ypair_fwd<T, NN>), dim3(blocks, 1, bt.nb), dim3(S::NT), ldsf, s, in0, out0, out1, t, bt); \
    }                                                                                                     \
  }
  KFBI_DISPATCH_N(N, KFBI_M)
#undef KFBI_M
  return hipGetLastError();
}

template <typename T>
hipError_t launch_axpy_scal(int64_t M, T* x, const T* d, const double* scal, int idx, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL((k_axpy_scal<T>), dim3(1024, 1, bt.nb), dim3(EW_NT), 0, s, M, x, d, scal, idx, bt);
  return hipGetLastError();
}

hipError_t launch_cg_coef(const double* rpart, int nr, const double* zpart, int nz, double* scal, int stokes,
                          int64_t M, hipStream_t s, const Bat& bt, double* hslot) {
  hipLaunchKernelGGL(k_cg_coef, dim3(1, 1, bt.nb), dim3(CG_NT), 0, s, rpart, nr, zpart, nz, scal, stokes, M, bt,
                     hslot);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nparts, int nper, double* scal, int op, int stokes, int64_t M,
                         hipStream_t s, double* out, const Bat& bt, double* hdst) {
  hipLaunchKernelGGL(k_reduce, dim3(1, 1, bt.nb), dim3(EW_NT), 0, s, partials, nparts, nper, scal, op, stokes, M, out,
                     bt, hdst);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dot_partials(int64_t M, const T* a, const T* b, double* partials, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_dot_partials<T>), dim3(nblocks), dim3(EW_NT), 0, s, M, a, b, partials);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_sum_partials(int64_t M, const T* a, double* partials, int nblocks, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL((k_sum_partials<T>), dim3(nblocks, 1, bt.nb), dim3(EW_NT), 0, s, M, a, partials, bt);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_add_scalar(int64_t M, T* a, const double* scal, int idx, double factor, hipStream_t s,
                             const Bat& bt) {
  hipLaunchKernelGGL((k_add_scalar<T>), dim3(ew_blocks(M), 1, bt.nb), dim3(256), 0, s, M, a, scal, idx, factor, bt);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_fill(int64_t n, T* a, T v, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL((k_fill<T>), dim3(ew_blocks(n), 1, bt.nb), dim3(256), 0, s, n, a, v, bt);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_axpby(int64_t n, T* y, double a, const T* x, double b, hipStream_t s) {
  hipLaunchKernelGGL((k_axpby<T>), dim3(ew_blocks(n)), dim3(256), 0, s, n, y, a, x, b);
  return hipGetLastError();
}


hipError_t launch_refine_prep(int64_t M, const double* F, float* r32, double* partials, int nparts, hipStream_t s,
                              const Bat& bt) {
  hipLaunchKernelGGL(k_refine_prep, dim3(nparts, 1, bt.nb), dim3(EW_NT), 0, s, M, F, r32, partials, bt);
  return hipGetLastError();
}
hipError_t launch_refine_residual(bool first, int N, double h, double mu, double c, const double* u, const double* p,
                                  const float* x32, const double* F, const double* shift, double* un, double* pn,
                                  float* r32, double* partials, int nparts, hipStream_t s, const Bat& bt,
                                  bool norms_only, const uint8_t* fmask) {
  if (nparts % 8) return hipErrorInvalidValue;  // XCD-aware chunking needs a multiple of 8 blocks
  if (norms_only && !first) return hipErrorInvalidValue;
  if (norms_only)
    hipLaunchKernelGGL((k_refine_residual<true, false>), dim3(nparts, 1, bt.nb), dim3(EW_NT), 0, s, N, h, mu, c, u, p,
                       x32, F, shift, un, pn, r32, partials, bt, fmask);
  else if (first)
    hipLaunchKernelGGL((k_refine_residual<true, true>), dim3(nparts, 1, bt.nb), dim3(EW_NT), 0, s, N, h, mu, c, u, p,
                       x32, F, shift, un, pn, r32, partials, bt, fmask);
  else
    hipLaunchKernelGGL((k_refine_residual<false, true>), dim3(nparts, 1, bt.nb), dim3(EW_NT), 0, s, N, h, mu, c, u,
                       p, x32, F, shift, un, pn, r32, partials, bt, fmask);
  return hipGetLastError();
}

static inline int gb(int64_t n) { return (int)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

hipError_t launch_fit_jump(int64_t T, const int64_t* nb_ptr, const int32_t* nb_idx, const double* fitw,
                           const double* jmap, const double* jfmap, const double* Fj, const double* phi,
                           const int64_t* cp_of, double* jumps, double* fitvals, hipStream_t s, const Bat& bt) {
  if (bt.act) return hipErrorInvalidValue;  // every right-hand side of a batch takes part
  hipLaunchKernelGGL(k_fit_jump, dim3(gb(T * FJ_LANES), 1, (bt.nb + FJ_RHS - 1) / FJ_RHS), dim3(256), 0, s, T, nb_ptr,
                     nb_idx, fitw, jmap, jfmap, Fj, phi, cp_of, jumps, fitvals, bt);
  return hipGetLastError();
}
hipError_t launch_interp_jump(int64_t n, const int64_t* cp_target, const double* fitvals, const double* emap,
                              const double* efmap, const double* Fj, double* ejump, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL(k_interp_jump, dim3(gb(3 * n), 1, bt.nb), dim3(256), 0, s, n, cp_target, fitvals, emap, efmap, Fj,
                     ejump, bt);
  return hipGetLastError();
}
hipError_t launch_correct(int64_t nirr, const int64_t* irr_node, const int64_t* irr_ptr, const int32_t* arm_t,
                          const int8_t* arm_o, const double* arm_a, const double* jumps, double* F, hipStream_t s,
                          float* r32, int64_t M, double* partials, int nparts, const Bat& bt) {
  const int blocks = r32 ? nparts : gb(nirr);
  if (r32 && (nparts < 1 || !partials)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_correct, dim3(blocks, 1, bt.nb), dim3(EW_NT), 0, s, nirr, irr_node, irr_ptr, arm_t, arm_o, arm_a,
                     jumps, F, r32, M, partials, bt);
  return hipGetLastError();
}
hipError_t launch_interp(int64_t n, const int64_t* idx, const double* w, const double* u, const double* ejump,
                         double* out, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL(k_interp, dim3(gb(3 * n), 1, bt.nb), dim3(256), 0, s, n, idx, w, u, ejump, out, bt);
  return hipGetLastError();
}
hipError_t launch_interp_x32(int64_t n, const int64_t* idx, const double* w, const float* x32, int N,
                             const double* ejump, double* out, hipStream_t s, const Bat& bt) {
  if (N < 2 || (N & (N - 1))) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_interp_x32, dim3(gb(3 * n), 1, bt.nb), dim3(256), 0, s, n, idx, w, x32, __builtin_ctz(N),
                     ejump, out, bt);
  return hipGetLastError();
}
hipError_t launch_stab(int64_t n, const int64_t* ptr, const int32_t* idx, const double* sw, const double* a,
                       const double* phi, double* out, hipStream_t s, const Bat& bt) {
  hipLaunchKernelGGL(k_stab, dim3(gb(3 * n), 1, bt.nb), dim3(256), 0, s, n, ptr, idx, sw, a, phi, out, bt);
  return hipGetLastError();
}
hipError_t launch_stab_T(int64_t n, const int64_t* ptr, const int32_t* row, const double* sw, const double* a,
                         const double* w, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_stab_T, dim3(gb(3 * n)), dim3(256), 0, s, n, ptr, row, sw, a, w, out);
  return hipGetLastError();
}
hipError_t launch_interp8(int64_t m, const int64_t* idx, const double* w, const double* u, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_interp8, dim3(gb(3 * m)), dim3(256), 0, s, m, idx, w, u, out);
  return hipGetLastError();
}
hipError_t launch_interp_T(int64_t nnode, const int64_t* ptr, const int64_t* node, const int32_t* row,
                           const double* w, const double* wbar, double* ubar, hipStream_t s) {
  hipLaunchKernelGGL(k_interp_T, dim3(gb(nnode)), dim3(256), 0, s, nnode, ptr, node, row, w, wbar, ubar);
  return hipGetLastError();
}
hipError_t launch_correct_T(int64_t T, const int64_t* ptr, const int64_t* node, const int8_t* slot, const double* a,
                            const double* Fbar, double* jbar, hipStream_t s) {
  hipLaunchKernelGGL(k_correct_T, dim3(gb(T)), dim3(256), 0, s, T, ptr, node, slot, a, Fbar, jbar);
  return hipGetLastError();
}
hipError_t launch_jump_T(int64_t T, const int64_t* cp_of, const double* jmap, const double* emap,
                         const double* jbar, const double* wbar, double* fitbar, hipStream_t s) {
  hipLaunchKernelGGL(k_jump_T, dim3(gb(T)), dim3(256), 0, s, T, cp_of, jmap, emap, jbar, wbar, fitbar);
  return hipGetLastError();
}
hipError_t launch_fit_T(int64_t n, const int64_t* ptr, const int64_t* entry, const int32_t* target,
                        const double* fitw, const double* fitbar, double* phibar, hipStream_t s) {
  hipLaunchKernelGGL(k_fit_T, dim3(gb(n)), dim3(256), 0, s, n, ptr, entry, target, fitw, fitbar, phibar);
  return hipGetLastError();
}
hipError_t launch_export_u(int N, const double* u_int, double* u_ext, hipStream_t s) {
  hipLaunchKernelGGL(k_export_u, dim3(ew_blocks(3LL * (N + 1) * N * N)), dim3(256), 0, s, N, u_int, u_ext);
  return hipGetLastError();
}
hipError_t launch_import_u(int N, const double* u_ext, double* u_int, hipStream_t s) {
  hipLaunchKernelGGL(k_import_u, dim3(ew_blocks(3LL * N * N * N)), dim3(256), 0, s, N, u_ext, u_int);
  return hipGetLastError();
}
hipError_t launch_scatter_add(int64_t n, const int64_t* idx, const double* v, double* F, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter_add, dim3(gb(n)), dim3(256), 0, s, n, idx, v, F);
  return hipGetLastError();
}
template <typename Ti, typename To>
hipError_t launch_convert(int64_t n, const Ti* in, To* out, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<Ti, To>), dim3(ew_blocks(n)), dim3(256), 0, s, n, in, out);
  return hipGetLastError();
}
template hipError_t launch_convert<double, float>(int64_t, const double*, float*, hipStream_t);
template hipError_t launch_convert<float, double>(int64_t, const float*, double*, hipStream_t);
template hipError_t launch_convert<double, double>(int64_t, const double*, double*, hipStream_t);

hipError_t launch_check_finite(int64_t n, const double* a, int* flag, int tag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_finite, dim3(ew_blocks(n)), dim3(256), 0, s, n, a, flag, tag);
  return hipGetLastError();
}

// explicit instantiations
#define KFBI_INST(T)                                                                                                 \
  template hipError_t launch_pass<T>(int, int, int, const T*, T*, bool, const DevTables<T>&, hipStream_t,          \
                                     const Bat&, const uint8_t*, const uint8_t*, int);                               \
  template hipError_t launch_xmid<T>(int, T*, T*, T*, double, const DevTables<T>&, hipStream_t, const Bat&);         \
  template hipError_t launch_zfwd_cg<T>(int, int, T*, T*, T*, const T*, T*, T*, const double*, double*,               \
                                        const DevTables<T>&, hipStream_t, const Bat&);                               \
  template hipError_t launch_ypair<T>(int, bool, const T*, const T*, T*, T*, const DevTables<T>&, hipStream_t,       \
                                      const Bat&);                                                                   \
  template hipError_t launch_xfuse<T>(int, int, bool, const T*, T*, T*, double, const DevTables<T>&, hipStream_t,    \
                                      const Bat&);                                                                   \
  template hipError_t launch_zinv_cg<T>(int, const T*, const T*, T*, const T*, double, double*, const DevTables<T>&, \
                                        hipStream_t, const Bat&);                                                    \
  template hipError_t launch_axpy_scal<T>(int64_t, T*, const T*, const double*, int, hipStream_t, const Bat&);       \
  template hipError_t launch_dot_partials<T>(int64_t, const T*, const T*, double*, int, hipStream_t);                \
  template hipError_t launch_sum_partials<T>(int64_t, const T*, double*, int, hipStream_t, const Bat&);              \
  template hipError_t launch_add_scalar<T>(int64_t, T*, const double*, int, double, hipStream_t, const Bat&);        \
  template hipError_t launch_fill<T>(int64_t, T*, T, hipStream_t, const Bat&);                                       \
  template hipError_t launch_axpby<T>(int64_t, T*, double, const T*, double, hipStream_t);
KFBI_INST(float)
KFBI_INST(double)
template hipError_t launch_fill<int>(int64_t, int*, int, hipStream_t, const Bat&);

}  // namespace kfbi
