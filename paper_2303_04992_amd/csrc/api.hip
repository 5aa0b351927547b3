// C ABI of libkfbi: context, device data, the operator evaluation pipeline, its transpose,
// mixed-precision refinement and the GMRES boundary-value solve.
//
// One evaluation (Algorithm 1 step 2 of the paper):
//   fit + jumps (per crossing)  ->  correction scatter into the MAC right-hand side
//   ->  MAC solve (spectral Schur-complement CG, velocity back-substitution)
//   ->  ten-node interpolation with the jump term  =  K phi.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/kfbi.h"
#include "kernels.h"
#include "setup.h"
#include "trig.h"

using namespace kfbi;

// Device scratch of kfbi_eval_noalloc: the per-call work buffers of one evaluation (MAC solver
// fields, right-hand side, grid solution, surface-stage values, partial sums) are carved from
// this array instead of the context's own workspaces.  Every device the library runs on holds
// one copy (KFBI_NOALLOC_MAX_BYTES) until the process ends.  In host code the array's name is
// only a stand-in: its device address on each device comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[KFBI_NOALLOC_MAX_BYTES];

namespace {

thread_local std::string g_create_error;

// device address of `scratch` per device, looked up once per device with that device current
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

void* scratch_address(int dev) {
  if (dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

struct DevErr {
  std::string msg;
};

#define HIPCHK(expr)                                                                                  \
  do {                                                                                                \
    hipError_t _e = (expr);                                                                           \
    if (_e != hipSuccess)                                                                             \
      throw DevErr{std::string(#expr) + ": " + hipGetErrorString(_e) + " (" + std::to_string(__LINE__) + ")"}; \
  } while (0)

template <typename T>
T* dalloc(size_t n, std::vector<void*>& owned) {
  void* p = nullptr;
  if (n == 0) n = 1;
  hipError_t e = hipMalloc(&p, n * sizeof(T));
  if (e != hipSuccess) throw DevErr{"hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed"};
  owned.push_back(p);
  return static_cast<T*>(p);
}

template <typename T>
T* dupload(const std::vector<T>& v, std::vector<void*>& owned, hipStream_t s) {
  T* p = dalloc<T>(v.size(), owned);
  if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return p;
}

void dfree(void* p, std::vector<void*>& owned) {
  if (!p) return;
  auto it = std::find(owned.begin(), owned.end(), p);
  if (it != owned.end()) owned.erase(it);
  (void)hipFree(p);
}

// Stage timing of one call from HIP events on the call's stream (no synchronisation between
// stages): mark(k) starts stage k; after the call's final synchronisation collect() sums the
// intervals per stage into kfbi_info.ms_stage and the whole span into ms_total.
enum Stage { ST_JUMPS = 0, ST_CORRECT = 1, ST_RHS = 2, ST_CG = 3, ST_BACKSUB = 4, ST_INTERP = 5, ST_END = 6 };
struct StageClock {
  static constexpr int CAP = 192;
  hipEvent_t ev[CAP] = {};
  int stage[CAP] = {};
  int used = 0;
  void init() {
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  }
  void release() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  void mark(int st, hipStream_t s) {
    if (used < CAP - 1 || (st == ST_END && used < CAP)) {
      HIPCHK(hipEventRecord(ev[used], s));
      stage[used++] = st;
    }
  }
  void collect(kfbi_info* info) {
    if (info && used >= 2) {
      for (int i = 0; i + 1 < used; ++i) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
        if (stage[i] < ST_END) info->ms_stage[stage[i]] += ms;
      }
      float tot = 0;
      HIPCHK(hipEventElapsedTime(&tot, ev[0], ev[used - 1]));
      info->ms_total += tot;
    }
    used = 0;
  }
};

// Sequential carving of device buffers (256-byte aligned) from one region; with base ==
// nullptr it only measures the bytes the same carving needs.
struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0;
  template <typename T>
  T* take(size_t n) {
    const size_t off = (used + 255) & ~(size_t)255;
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    used = off + bytes;
    if (!base) return nullptr;
    if (used > size) throw std::invalid_argument("scratch region too small");
    return reinterpret_cast<T*>(base + off);
  }
};

// the work buffers of a MacSolver (everything a solve writes)
template <typename T>
struct SolverPtrs {
  T *Fh[3], *b, *x, *r, *d, *q, *A, *B, *A1, *B2, *B3;
  double *partials, *rpart, *scal;
};

// ---------------------------------------------------------------------------------------
// spectral MAC solver in precision T
// ---------------------------------------------------------------------------------------
template <typename T>
struct MacSolver {
  int N = 0;
  int64_t M = 0;
  int pde = 0;
  double mu = 1, c = 0;
  hipStream_t s = nullptr;
  DevTables<T> tb;
  T *Fh[3] = {nullptr, nullptr, nullptr}, *b = nullptr, *x = nullptr, *r = nullptr, *d = nullptr, *q = nullptr;
  T *A = nullptr, *B = nullptr, *A1 = nullptr, *B2 = nullptr, *B3 = nullptr;
  double* partials = nullptr;
  double* rpart = nullptr;  // partial r.r of the forward z pass
  double* scal = nullptr;
  double* host_rr = nullptr;  // pinned: two look-ahead slots of the 8 CG scalars (scal[0..7])
  double* host_rr_dev = nullptr;  // its device address (the coefficient kernel writes it)
  double* coef_slot = nullptr;    // slot of the iteration being queued (device address)
  StageClock* clock = nullptr;  // stage marks of the calling context
  void mark(int st) {
    if (clock) clock->mark(st, s);
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  int nparts_x = 0, nparts_z = 0, nparts_u = 1024;
  // live timing of one transform-pass kind with HIP events on the solver stream
  int prof_kind = -1, prof_axis = -1;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev;
  size_t prof_used = 0;
  int64_t prof_launches = 0;
  double prof_ms = 0;
  // algorithmic HBM bytes of the launches issued (one read or write per N^3 field touched, for
  // each right-hand side the launch serves)
  double bytes = 0;
  int nact = 1;
  void count(double fields) { bytes += fields * (double)M * sizeof(T) * nact; }
  // Batches (several right-hand sides in lockstep, see Bat): bt describes the call's batch;
  // act_live flags the right-hand sides a solve serves, act_cg those whose CG still iterates;
  // cur is the descriptor the launches use (live or CG flags), nact its active count.
  Bat bt, cur;
  int* act_live = nullptr;
  int* act_cg = nullptr;
  int rr_cap = 1;  // right-hand sides host_rr has room for
  // hi/lo bfloat16 fragments of the DCT-II matrix for the matrix-core pass (built on first use)
  void* gemm_cf = nullptr;
  void ensure_gemm(std::vector<void*>& owned) {
    if (gemm_cf) return;
    if (sizeof(T) != 4 || !gemm_pass_supported(N))
      throw std::invalid_argument("the matrix-core DCT-II pass needs a MIXED_FP32 context with N = 128, 256 or 512");
    gemm_cf = dupload(gemm_dct2_fragments(N), owned, s);
    HIPCHK(hipStreamSynchronize(s));
  }
  template <class Q>
  Q* at(Q* p, int r) const {
    return p ? reinterpret_cast<Q*>(reinterpret_cast<uintptr_t>(p) + (uint64_t)r * (uint64_t)bt.A) : p;
  }

  void init(int N_, double h, int pde_, double mu_, double c_, hipStream_t s_, std::vector<void*>& owned) {
    N = N_;
    M = (int64_t)N * N * N;
    pde = pde_;
    mu = mu_;
    c = c_;
    s = s_;
    // tables (computed in float64, stored in T)
    std::vector<T> tw(2 * N), tw2(4 * N), mk(2 * N), sc(N), isc(N);
    for (int k = 0; k < N; ++k) {
      tw[2 * k] = T(std::cos(2 * M_PI * k / N));
      tw[2 * k + 1] = T(-std::sin(2 * M_PI * k / N));
      mk[2 * k] = T(std::cos(M_PI * k / (2.0 * N)));
      mk[2 * k + 1] = T(-std::sin(M_PI * k / (2.0 * N)));
      double sk = (k == 0) ? std::sqrt(1.0 / N) : std::sqrt(2.0 / N);
      sc[k] = T(sk);
      isc[k] = T(1.0 / sk);
    }
    for (int k = 0; k < 2 * N; ++k) {
      tw2[2 * k] = T(std::cos(2 * M_PI * k / (2.0 * N)));
      tw2[2 * k + 1] = T(-std::sin(2 * M_PI * k / (2.0 * N)));
    }
    std::vector<double> sig(N), sig2s(N);
    for (int k = 0; k < N; ++k) {
      sig[k] = 2.0 / h * std::sin(M_PI * k / (2.0 * N));
      double s1 = 2.0 / h * std::sin(M_PI * (k + 1) / (2.0 * N));
      sig2s[k] = s1 * s1;
    }
    tb.tw = dupload(tw, owned, s);
    tb.tw2 = dupload(tw2, owned, s);
    tb.mk = dupload(mk, owned, s);
    tb.sc = dupload(sc, owned, s);
    tb.isc = dupload(isc, owned, s);
    tb.s0 = sc[0];
    tb.s1 = sc[N > 1 ? 1 : 0];
    tb.is0 = isc[0];
    tb.is1 = isc[N > 1 ? 1 : 0];
    tb.sig = dupload(sig, owned, s);
    tb.sig2s = dupload(sig2s, owned, s);
    std::vector<T> sg2t(N), sg2st(N);
    for (int k = 0; k < N; ++k) {
      sg2t[k] = T(sig[k] * sig[k]);
      sg2st[k] = T(sig2s[k]);
    }
    tb.sg2 = dupload(sg2t, owned, s);
    tb.sg2s = dupload(sg2st, owned, s);
    for (int m = 0; m < 3; ++m) Fh[m] = dalloc<T>(M, owned);
    b = dalloc<T>(M, owned);
    x = dalloc<T>(M, owned);
    r = dalloc<T>(M, owned);
    d = dalloc<T>(M, owned);
    q = dalloc<T>(M, owned);
    A = dalloc<T>(M, owned);
    B = dalloc<T>(M, owned);
    A1 = dalloc<T>(M, owned);
    B2 = dalloc<T>(M, owned);
    B3 = dalloc<T>(M, owned);
    nparts_x = zinv_blocks(N, sizeof(T));
    nparts_z = zfwd_blocks(N, sizeof(T));
    partials = dalloc<double>(std::max(4 * nparts_x, nparts_u), owned);
    rpart = dalloc<double>(nparts_z, owned);
    scal = dalloc<double>(16, owned);
    HIPCHK(hipHostMalloc((void**)&host_rr, 16 * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostGetDevicePointer((void**)&host_rr_dev, host_rr, 0));
    HIPCHK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  }
  void release() {
    if (host_rr) (void)hipHostFree(host_rr);
    host_rr = nullptr;
    host_rr_dev = nullptr;
    for (auto& e : prof_ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    prof_ev.clear();
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    ev[0] = ev[1] = nullptr;
  }

  SolverPtrs<T> ptrs() const { return {{Fh[0], Fh[1], Fh[2]}, b, x, r, d, q, A, B, A1, B2, B3, partials, rpart, scal}; }
  void set(const SolverPtrs<T>& w) {
    for (int m = 0; m < 3; ++m) Fh[m] = w.Fh[m];
    b = w.b, x = w.x, r = w.r, d = w.d, q = w.q, A = w.A, B = w.B, A1 = w.A1, B2 = w.B2, B3 = w.B3;
    partials = w.partials, rpart = w.rpart, scal = w.scal;
  }
  // the same buffers carved from an arena (sizes as in init)
  SolverPtrs<T> carve(Arena& a) const {
    SolverPtrs<T> w;
    for (auto& f : w.Fh) f = a.take<T>(M);
    for (T** f : {&w.b, &w.x, &w.r, &w.d, &w.q, &w.A, &w.B, &w.A1, &w.B2, &w.B3}) *f = a.take<T>(M);
    w.partials = a.take<double>(std::max(4 * nparts_x, nparts_u));
    w.rpart = a.take<double>(nparts_z);
    w.scal = a.take<double>(16);
    return w;
  }

  // launch under HIP events when kernel id (and axis, for the single passes) is being timed
  template <class F>
  void timed(bool on, F&& launch) {
    if (on) {
      if (prof_used == prof_ev.size()) {
        hipEvent_t a, b;
        HIPCHK(hipEventCreate(&a));
        HIPCHK(hipEventCreate(&b));
        prof_ev.push_back({a, b});
      }
      HIPCHK(hipEventRecord(prof_ev[prof_used].first, s));
    }
    HIPCHK(launch());
    if (on) HIPCHK(hipEventRecord(prof_ev[prof_used++].second, s));
  }
  void pass(int kind, int axis, const T* in, T* out, bool acc = false) {
    count(acc ? 3 : 2);
    timed(kind == prof_kind && (prof_axis < 0 || axis == prof_axis) && !acc,
          [&] { return launch_pass<T>(N, kind, axis, in, out, acc, tb, s, cur); });
  }
  // Sparse right-hand side (set by the caller for one solve, else null): component m of Fu is
  // zero outside the z-pencils flagged with bit m in sp_pmask (sp_xmask: or over y); sp_zread[m],
  // sp_yread[m]: the shares of the z and y tiles of component m that hold such a pencil
  const uint8_t* sp_pmask = nullptr;
  const uint8_t* sp_xmask = nullptr;
  double sp_zread[3] = {1, 1, 1}, sp_yread[3] = {1, 1, 1};
  void pass_sparse(int kind, int axis, const T* in, T* out, int m) {
    const double share = !sp_pmask ? 1.0 : axis == 2 ? sp_zread[m] : sp_yread[m];
    count(1 + share);  // the tiles read, and every tile written
    timed(kind == prof_kind && (prof_axis < 0 || axis == prof_axis),
          [&] { return launch_pass<T>(N, kind, axis, in, out, false, tb, s, cur, sp_pmask, sp_xmask, m); });
  }
  // algorithmic HBM bytes of one launch of kernel id (one read and one write per field touched)
  double kernel_bytes(int id) const {
    const double f = (double)M * sizeof(T);
    switch (id) {
      case KFBI_K_XMID: return 6 * f;  // three fields read and written
      case KFBI_K_ZFWD: return 9 * f;  // x, r, d, q read; x, r, d, A, B written
      case KFBI_K_ZINV: return 4 * f;  // A, B, d read; q written
      case KFBI_K_YFWD: return 3 * f;  // A read; A1, B2 written
      case KFBI_K_YINV: return 3 * f;  // A1, B2 read; A written
      case KFBI_K_GEMM_X: return 2 * f;  // one field read and written
      default: return 2 * f;           // single transform pass
    }
  }
  // accumulate the recorded launch durations (call after the stream has drained)
  void prof_collect() {
    for (size_t i = 0; i < prof_used; ++i) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, prof_ev[i].first, prof_ev[i].second));
      prof_ms += ms;
      ++prof_launches;
    }
    prof_used = 0;
  }
  // v -= mean v; the sum of v is left in scal[keep] when keep >= 0
  void project_mean(T* v, int keep = -1) {
    count(3);
    HIPCHK(launch_sum_partials<T>(M, v, partials, nparts_u, s, cur));
    HIPCHK(launch_reduce(partials, nparts_u, 1, scal, R_SUM, 1, M, s, keep >= 0 ? scal + keep : nullptr, cur));
    HIPCHK(launch_add_scalar<T>(M, v, scal, keep >= 0 ? keep : 5, -1.0 / (double)M, s, cur));
  }

  // S p for the CG direction d (q = S d); the updates of x, r (previous iteration) and of
  // d = r + beta d_old are formed in the first pass
  // C_0 = DCT_x DST_y DST_z, C_1 = DST_x DCT_y DST_z, C_2 = DST_x DST_y DCT_z (orthonormal);
  // order z, y, [x fused with the weights], y, z
  void zfwd(int mode = ZF_FUSED) {
    count(mode == ZF_FUSED ? 9 : mode == ZF_FIRST ? 6 : 3);
    timed(prof_kind == KFBI_K_ZFWD && mode == ZF_FUSED,
          [&] { return launch_zfwd_cg<T>(N, mode, x, r, d, q, A, B, scal, rpart, tb, s, cur); });
  }
  void yfwd() {
    count(3);
    timed(prof_kind == KFBI_K_YFWD, [&] { return launch_ypair<T>(N, false, A, A, A1, B2, tb, s, cur); }); }
  void xmid() {
    count(6);
    timed(prof_kind == KFBI_K_XMID, [&] { return launch_xmid<T>(N, A1, B2, B3, mu, tb, s, cur); }); }
  void yinv() {
    count(3);
    timed(prof_kind == KFBI_K_YINV, [&] { return launch_ypair<T>(N, true, A1, B2, A, A, tb, s, cur); }); }
  void zinv() {
    count(4);
    timed(prof_kind == KFBI_K_ZINV, [&] { return launch_zinv_cg<T>(N, A, B, q, d, c, partials, tb, s, cur); });
  }
  void cg_iteration(bool first) {
    zfwd(first ? ZF_FIRST : ZF_FUSED);  // x, r of the last step; d = r + beta d; A = DST_z d; B = DCT_z d
    // y passes, ordered so that the x pass starts with the components written last (still in the
    // 256 MB last-level cache): float32 runs component 2 first and the x pass takes components
    // 0, 1, 2; float64 runs components 0, 1 first and the x pass takes 2, 1, 0 (measured at 256^3)
    constexpr bool b3_first = sizeof(T) == 4;
    if (b3_first) pass(DST2, 1, B, B3);  // component 2
    yfwd();                               // components 0, 1: A1 = DST_y A, B2 = DCT_y A
    if (!b3_first) pass(DST2, 1, B, B3);
    xmid();                               // x: forward, weight sigma^2 / Lambda, inverse (all components)
    yinv();                               // A = DST_y^T A1 + DCT_y^T B2 (components 0 and 1 share DST_z)
    pass(DST3, 1, B3, B);
    zinv();                // q = DST_z^T A + DCT_z^T B + c d, partial dots
    HIPCHK(launch_cg_coef(rpart, nparts_z, partials, nparts_x, scal, 1, M, s, cur, coef_slot));  // mean-zero iterates
  }

  // Solve A_u u + G p = F_u, D u + c p = F_p (Stokes: D u = F_p - mean F_p, mean p = 0).
  // Fu: 3 fields (internal layout, face 0 ignored), Fp: 1 field.  Returns CG iterations or
  // -1 if maxit was reached.
  // Batch set-up: right-hand sides r with live[r] != 0 take part (null: all); the flags go to
  // the device before the solve's first launch (pageable source: copied at the call).
  void set_live(const std::vector<char>* live, int& nlive) {
    nlive = bt.nb;
    if (bt.nb == 1) {
      cur = bt;
      nact = 1;
      return;
    }
    std::vector<int> f(bt.nb, 1);
    if (live) {
      nlive = 0;
      for (int r = 0; r < bt.nb; ++r) nlive += (f[r] = (*live)[r] ? 1 : 0);
    }
    HIPCHK(hipMemcpyAsync(act_live, f.data(), bt.nb * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(act_cg, f.data(), bt.nb * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));  // the pageable source is read before f goes out of scope
  }
  Bat with_act(const int* act) const {
    Bat b = bt;
    b.act = bt.nb > 1 ? act : nullptr;
    return b;
  }

  // Solve A_u u + G p = F_u, D u + c p = F_p (Stokes: D u = F_p - mean F_p, mean p = 0).
  // Fu: 3 fields (internal layout, face 0 ignored), Fp: 1 field.  Returns the CG iterations
  // (the largest over a batch) or -1 if maxit was reached.  Batches (bt.nb > 1) solve every
  // live right-hand side in lockstep; each stops by the same rule, at the same iteration, as
  // its own solve would (its flag in act_cg then skips it), and its iteration count goes to
  // its[r].
  // mean_free = false (Stokes only): the mean of p is left as the iterations made it (a
  // rounding drift; the velocity does not depend on it), for callers that project it later
  int solve(const T* Fu, const T* Fp, T* u, T* p, double rtol, int maxit, const std::vector<char>* live = nullptr,
            std::vector<int>* its = nullptr, bool mean_free = true) {
    const int NB = bt.nb;
    // the CG iterate x lives in the caller's p itself (no copy after the solve)
    struct XGuard {
      T*& x;
      T* own;
      ~XGuard() { x = own; }
    } xguard{x, x};
    if (p) x = p;
    int nlive = 1;
    set_live(live, nlive);
    auto is_live = [&](int r) { return !live || (*live)[r]; };
    cur = with_act(act_live);
    nact = nlive;
    // 1.-2. b = P(F_p - sum_m C_m^T [sigma/Lambda_m] T_m F_m).  Per component: T_m along z and
    // y, then the fused x pass keeps Fh[m] = T_m F_m and leaves C_m,x^T of the weighted
    // spectrum; the y and z inverses of the three components are shared as in the matvec.
    T* H[3] = {A1, B2, B3};
    mark(ST_RHS);
    for (int m = 0; m < 3; ++m) {
      pass_sparse(m == 2 ? DST1 : DST2, 2, Fu + m * M, Fh[m], m);
      pass_sparse(m == 1 ? DST1 : DST2, 1, Fh[m], Fh[m], m);
      HIPCHK(launch_xfuse<T>(N, m, false, Fh[m], Fh[m], H[m], mu, tb, s, cur));
      count(3);
    }
    HIPCHK(launch_ypair<T>(N, true, A1, B2, A, A, tb, s, cur));       // A = DST_y^T H0 + DCT_y^T H1
    pass(DST3, 1, B3, B);                                             // B = DST_y^T H2
    HIPCHK(launch_zinv_cg<T>(N, A, B, b, Fp, 1.0, partials, tb, s, cur));  // b = DST_z^T A + DCT_z^T B + F_p
    count(3 + 4);
    // Both PDEs iterate on mean-zero pressures.  S = S_0 + cI with S_0 1 = 0 (G annihilates
    // constants, sigma_0 = 0) and S_0 symmetric, so the mean of S p is c mean(p): for Navier
    // (c > 0) the constant mode, whose eigenvalue c = 1/(lambda + mu) is the smallest of S and
    // grows the iteration count as nu -> 1/2, is solved exactly, mean(p) = mean(b) / c, and CG
    // runs on the mean-zero part.  Stokes (c = 0): P b, mean(p) = 0.
    // sum of b (kept in scal[9]) from the partial sums of the z inverse pass that formed it; the
    // first forward z pass of the CG subtracts the mean
    HIPCHK(launch_reduce(partials, nparts_x, 4, scal, R_SUM1, 1, M, s, scal + 9, cur));
    // 3. CG on S x = b.  Iteration k forms x_k, r_k (with alpha_{k-1}) and d_k in its first
    // pass, so x lags one step until the final x += alpha d.
    // The residual starts as b itself (b is not needed afterwards: the buffers swap roles), and
    // the first iteration's coefficient kernel leaves r_0.r_0 = |b|^2 in scal[7], read at the
    // first check (no synchronisation before the first iterations are queued; b = 0 converges
    // at that check with x = 0).
    mark(ST_CG);
    std::swap(r, b);  // x = 0 is set by the first forward z pass
    // Stop test.  Iteration k leaves in scal[7] the r_k.r_k that its forward z pass summed over
    // the updated residual r_k, and in scal[0] the recurrence estimate of |r_{k+1}|^2 (used
    // for beta only: it assumes the conjugacy of d_k and d_{k-1}).  With one iteration of
    // look-ahead, iteration k+1 is queued before the values of k are read.  A solve has
    // converged when the summed r_k.r_k is below the threshold, or when the estimate of
    // |r_{k+1}|^2 is and the r_{k+1}.r_{k+1} that the queued iteration k+1 sums confirms it
    // (a non-positive or drifted estimate alone never stops the solve).  Its pending
    // x += alpha d (alpha of the queued iteration) is issued right then.
    // host_rr: two look-ahead slots, each 8 scalars per right-hand side
    auto slot = [&](int i, int rhs) { return host_rr + 8 * ((i & 1) * NB + rhs); };
    std::vector<double> bb(NB, 0.0);
    std::vector<char> done(NB, 0);
    int it = 0, ndone = 0;
    for (int rr = 0; rr < NB; ++rr)
      if (!is_live(rr)) done[rr] = 1, ++ndone;
    cur = with_act(act_cg);
    auto nan_check = [&](double v) {
      if (std::isnan(v)) throw DevErr{"NaN in the Schur CG residual"};
    };
    // Without a mean projection between the solve and the back-substitution (mean_free false,
    // c = 0), the pending x += alpha d of a finished right-hand side is left to the first pass
    // of the back-substitution (its x, d and alpha stay untouched: later iterations skip it).
    const bool defer_final = !mean_free && c == 0;
    auto finish = [&](int rr) {  // right-hand side rr has converged: its pending update, and out
      done[rr] = 1;
      ++ndone;
      --nact;
      if (its) (*its)[rr] = it;
      Bat one = bt;
      one.nb = 1;
      one.act = nullptr;
      if (!defer_final) {
        HIPCHK(launch_axpy_scal<T>(M, at(x, rr), at(d, rr), at(scal, rr), 1, s, one));  // x += alpha d
        bytes += 3.0 * M * sizeof(T);
      }
      if (NB > 1) HIPCHK(launch_fill<int>(1, act_cg + rr, 0, s));
    };
    while (ndone < NB && it < maxit) {
      // the coefficient kernel writes scal[0] and scal[7] of each right-hand side straight into
      // the iteration's host slot (a copy operation there would put a gap of about 20 us
      // between the iterations' kernels)
      coef_slot = host_rr_dev + 8 * ((it & 1) * NB);
      cg_iteration(it == 0);
      coef_slot = nullptr;
      HIPCHK(hipEventRecord(ev[it & 1], s));
      ++it;
      if (it >= 2) {
        const int k = it - 2;
        HIPCHK(hipEventSynchronize(ev[k & 1]));
        std::vector<int> confirm, conv_now;
        for (int rr = 0; rr < NB; ++rr) {
          if (done[rr]) continue;
          if (k == 0) bb[rr] = slot(0, rr)[7];
          const double thr = rtol * rtol * bb[rr], est = slot(k, rr)[0], tru = slot(k, rr)[7];
          nan_check(est);
          nan_check(tru);
          if (!(tru > thr))
            conv_now.push_back(rr);
          else if (!(est > thr))
            confirm.push_back(rr);
        }
        if (!confirm.empty()) {
          HIPCHK(hipEventSynchronize(ev[(k + 1) & 1]));
          for (int rr : confirm) {
            nan_check(slot(k + 1, rr)[7]);
            if (!(slot(k + 1, rr)[7] > rtol * rtol * bb[rr])) conv_now.push_back(rr);
          }
        }
        for (int rr : conv_now) finish(rr);
      }
    }
    bool conv = ndone == NB;
    if (!conv && it > 0) {  // maxit reached: the last iteration's summed residual decides
      HIPCHK(hipEventSynchronize(ev[(it - 1) & 1]));
      conv = true;
      for (int rr = 0; rr < NB; ++rr) {
        if (done[rr]) continue;
        if (it == 1) bb[rr] = slot(0, rr)[7];
        nan_check(slot(it - 1, rr)[7]);
        const bool ok = !(slot(it - 1, rr)[7] > rtol * rtol * bb[rr]);
        finish(rr);
        conv = conv && ok;
      }
    }
    cur = with_act(act_live);
    nact = nlive;
    if (mean_free || c > 0) project_mean(x);
    if (c > 0) {
      HIPCHK(launch_add_scalar<T>(M, x, scal, 9, 1.0 / ((double)M * c), s, cur));  // + mean(b) / c
      count(2);
    }
    // 4. velocity back-substitution u_m = T_m^T [(T_m F_m + sigma C_m p) / Lambda_m]: C_m p along
    // z and y shared as in the matvec, then per component the fused x pass and the y, z inverses
    // A = DST_z p, B = DCT_z p
    mark(ST_BACKSUB);
    if (defer_final) {  // x += alpha d, written back, and its transforms
      HIPCHK(launch_zfwd_cg<T>(N, ZF_FINAL, nullptr, x, d, nullptr, A, B, scal, nullptr, tb, s, cur));
      count(2);
    } else {
      HIPCHK(launch_zfwd_cg<T>(N, ZF_PLAIN, nullptr, x, nullptr, nullptr, A, B, nullptr, nullptr, tb, s, cur));
    }
    if (sizeof(T) == 4) pass(DST2, 1, B, B3);                         // C_2 along y (order as in the matvec)
    HIPCHK(launch_ypair<T>(N, false, A, A, A1, B2, tb, s, cur));     // C_0, C_1 along y
    count(3 + 3);
    if (sizeof(T) != 4) pass(DST2, 1, B, B3);
    for (int m = 0; m < 3; ++m) {
      T* um = u + m * M;
      HIPCHK(launch_xfuse<T>(N, m, true, H[m], Fh[m], um, mu, tb, s, cur));
      count(3);
      pass(m == 1 ? DST1 : DST3, 1, um, um);
      pass(m == 2 ? DST1 : DST3, 2, um, um);
    }
    cur = bt;
    nact = 1;
    if (prof_used) {
      HIPCHK(hipStreamSynchronize(s));
      prof_collect();
    }
    return conv ? it : -1;
  }
};

}  // namespace

// ---------------------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------------------
struct kfbi_plan {
  kfbi_config cfg;
  Setup S;
};

struct kfbi_ctx {
  kfbi_config cfg;
  Setup S;
  std::string err;
  int dev = 0;  // device current at kfbi_create
  hipStream_t s = nullptr;
  std::vector<void*> owned;
  int64_t M = 0;
  // surface maps
  int64_t *nb_ptr, *irr_node, *irr_ptr, *itp_idx, *cp_target, *cp_of, *uT_ptr, *uT_node, *cT_ptr, *cT_node;
  int64_t *fT_ptr, *fT_entry, *sv_ptr, *svT_ptr;
  int32_t *nb_idx, *arm_t, *uT_row, *fT_target, *sv_idx, *svT_row;
  double *stab_a, *sv_w, *svT_w;
  int8_t *arm_o, *cT_slot;
  double *fitw, *jmap, *jfmap, *emap, *efmap, *arm_a, *itp_w, *uT_w, *cT_a;
  // work
  double *jumps, *fitvals, *ejump, *F, *u, *p, *jbar, *fitbar;
  // body force of the last kfbi_solve_bvp with f != NULL: the force jumps at the crossings (Fj)
  // and the volume values at the interior nodes; has_force covers both (set together)
  bool has_force = false;
  double* Fj = nullptr;
  double* vol_val = nullptr;
  int64_t* vol_idx = nullptr;
  int64_t nvol = 0, vol_cap = 0;
  // solvers
  MacSolver<double> s64;
  MacSolver<float> s32;
  bool mixed = false;
  // mixed refinement fields (float64 and float32)
  double* ru = nullptr;  // spare float64 iterate of the refinement
  float *r32 = nullptr, *x32 = nullptr;
  float* r32b = nullptr;  // residual of the rounds after the first (r32 keeps the first right-hand side)
  // r32 is zero outside the irregular nodes (the correction pass then assigns them), and
  // r32_ready: r32 = float32(F) and rpart holds its partial sums, written by the last assembly
  bool r32_clean = false, r32_ready = false;
  double* rscal = nullptr;
  double* rpart = nullptr;
  // GMRES
  double *V = nullptr, *H = nullptr, *gtmp = nullptr;
  // interior probes (trilinear interpolation on T^1..T^3) and the transposed map
  int64_t nprobe = 0, nprobe_nodes = 0;
  int64_t *pr_idx = nullptr, *prT_ptr = nullptr, *prT_node = nullptr;
  int32_t* prT_row = nullptr;
  double *pr_w = nullptr, *prT_w = nullptr;
  int gm_max = 0;
  double* pbar = nullptr;  // probe cotangent pulled back to the density (kfbi_solve_bvp_adjoint)
  kfbi_info last;
  // algorithmic HBM bytes of the surface stages of one evaluation (fit + jumps, corrections,
  // interpolation), from the map sizes; refinement passes are counted as they run
  double bytes_jumps = 0, bytes_correct = 0, bytes_interp = 0, bytes_extra = 0;
  // F is zero outside the irregular nodes (the correction pass then assigns those and no clear
  // of the 4 N^3 values is needed); false after any other writer of F
  bool f_clean = false;
  // the last mac_solve left its velocity in x32 (lean mixed solve; C->u and C->p not written)
  bool u_x32 = false;
  // per z-pencil flags of the components of F that can be nonzero while F is clean (the
  // irregular nodes): the refinement passes read F only there
  uint8_t* fmask = nullptr;
  double fmask_frac = 1;  // share of the (pencil, component) pairs flagged
  uint8_t* fxmask = nullptr;  // the flags or-ed over y, per plane x
  double fz_share[2][3] = {}, fy_share[3] = {};  // tile shares (float32, float64 z tiles; planes)
  // pinned host scalars written by kernels and read after a later synchronisation (hflag: the
  // tag of the current call's input check if it saw a non-finite value), their device
  // addresses, and the stage clock of a call
  double* hpin = nullptr;
  int* hflag = nullptr;
  double* hpin_dev = nullptr;
  int* hflag_dev = nullptr;
  int check_tag = 0;
  StageClock clock;
  // batched evaluations (kfbi_eval_batch): the current batch of the context-level launches, the
  // per-right-hand-side work arenas (bat_A bytes each) and their flags
  Bat bt;
  char* bat_base = nullptr;
  int64_t bat_A = 0;
  int bat_cap = 0, bat_clean = 0;
  int* bat_act = nullptr;  // 3 x bat_cap flags: the solver's live and CG flags, the refinement's
  double* hpin_bat = nullptr;  // pinned: |F| and |r| of each right-hand side (2 x bat_cap)
  double* hpin_bat_dev = nullptr;
  ~kfbi_ctx() {
    if (hpin) (void)hipHostFree(hpin);
    if (hflag) (void)hipHostFree(hflag);
    if (hpin_bat) (void)hipHostFree(hpin_bat);
    clock.release();
    s64.release();
    s32.release();
    for (void* q : owned) (void)hipFree(q);
    if (s && !cfg.stream) (void)hipStreamDestroy(s);
  }
};

static kfbi_config normalized(const kfbi_config* c) {
  kfbi_config r = *c;
  if (r.cg_rtol <= 0) r.cg_rtol = 1e-12;
  if (r.cg_maxit <= 0) r.cg_maxit = 2000;
  if (r.inner_rtol <= 0) r.inner_rtol = 1e-5;
  if (r.gmres_rtol <= 0) r.gmres_rtol = 1e-8;
  if (r.gmres_maxit <= 0) r.gmres_maxit = 200;
  return r;
}

static const char* validate(const kfbi_config* c) {
  if (!c) return "null config";
  int N = c->N;
  if (N < 16 || N > 512 || (N & (N - 1))) return "N must be a power of two in [16, 512]";
  if (!(c->hi > c->lo)) return "box must satisfy hi > lo";
  if (!(c->mu > 0) || !std::isfinite(c->mu)) return "mu must be positive";
  if (c->pde == KFBI_NAVIER && !(c->lambda + c->mu > 0)) return "lambda + mu must be positive";
  if (c->pde != KFBI_STOKES && c->pde != KFBI_NAVIER) return "unknown pde";
  if (c->precision != KFBI_FP64 && c->precision != KFBI_MIXED_FP32) return "unknown precision";
  if (c->shape.kind < KFBI_SPHERE || c->shape.kind > KFBI_TORUS) return "unknown shape";
  if (c->trace != KFBI_TRACE_INTERIOR && c->trace != KFBI_TRACE_AVERAGE) return "unknown trace form";
  return nullptr;
}

static kfbi_status status_of_setup(const std::string& e) {
  return e.rfind("GEOM:", 0) == 0 ? KFBI_EGEOM : KFBI_EINVAL;
}

extern "C" {

kfbi_status kfbi_plan_create(const kfbi_config* cfg, kfbi_plan** out);
void kfbi_plan_destroy(kfbi_plan* p);

kfbi_status kfbi_create(const kfbi_config* cfg_in, kfbi_ctx** out) {
  if (!out) return KFBI_EINVAL;
  *out = nullptr;
  if (const char* v = validate(cfg_in)) {
    g_create_error = v;
    return KFBI_EINVAL;
  }
  std::unique_ptr<kfbi_ctx> C(new kfbi_ctx());
  C->cfg = normalized(cfg_in);
  std::string e;
  try {
    e = build_setup(C->cfg, C->S);
  } catch (const std::exception& ex) {
    e = std::string("setup failed: ") + ex.what();
  }
  if (!e.empty()) {
    g_create_error = e;
    return status_of_setup(e);
  }
  try {
    Setup& S = C->S;
    if (C->cfg.stream)
      C->s = (hipStream_t)C->cfg.stream;
    else
      HIPCHK(hipStreamCreate(&C->s));
    hipStream_t s = C->s;
    auto& o = C->owned;
    HIPCHK(hipGetDevice(&C->dev));
    if (!scratch_address(C->dev)) throw DevErr{"hipGetSymbolAddress of the no-alloc scratch failed"};
    HIPCHK(hipHostMalloc((void**)&C->hpin, 16 * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&C->hflag, sizeof(int), hipHostMallocDefault));
    *C->hflag = 0;
    HIPCHK(hipHostGetDevicePointer((void**)&C->hpin_dev, C->hpin, 0));
    HIPCHK(hipHostGetDevicePointer((void**)&C->hflag_dev, C->hflag, 0));
    C->clock.init();
    C->M = S.M;
    C->nb_ptr = dupload(S.nb_ptr, o, s);
    C->nb_idx = dupload(S.nb_idx, o, s);
    C->fitw = dupload(S.fitw, o, s);
    {  // component-major on the device: consecutive crossings are adjacent for every (r, c)
      std::vector<double> jt(S.jmap.size());
      for (int64_t t = 0; t < S.T; ++t)
        for (int rc = 0; rc < 90; ++rc) jt[(int64_t)rc * S.T + t] = S.jmap[t * 90 + rc];
      C->jmap = dupload(jt, o, s);
    }
    C->jfmap = dupload(S.jfmap, o, s);
    std::vector<double> em(S.emap.begin(), S.emap.begin() + S.n * 54);
    std::vector<double> efm(S.emap.begin() + S.n * 54, S.emap.end());
    C->emap = dupload(em, o, s);
    C->efmap = dupload(efm, o, s);
    C->irr_node = dupload(S.irr_node, o, s);
    {  // per z-pencil (x, y): bit c set iff component c of F has an irregular node in the pencil
      std::vector<uint8_t> fm((size_t)S.N * S.N, 0);
      for (int64_t node : S.irr_node) {
        const int64_t c = node / S.M, cell = node % S.M;
        fm[(size_t)(cell / S.N)] |= (uint8_t)(1u << c);
      }
      int64_t bits = 0;
      for (uint8_t v : fm) bits += __builtin_popcount(v);
      C->fmask_frac = (double)bits / (4.0 * (double)fm.size());
      C->fmask = dupload(fm, o, s);
      // or over y of each plane x, and the shares of the z tiles (W pencils of one plane) and of
      // the planes that hold a flagged pencil, per velocity component
      std::vector<uint8_t> xm((size_t)S.N, 0);
      for (int x = 0; x < S.N; ++x)
        for (int y = 0; y < S.N; ++y) xm[x] |= fm[(size_t)x * S.N + y];
      C->fxmask = dupload(xm, o, s);
      for (int m = 0; m < 3; ++m) {
        int64_t planes = 0;
        for (uint8_t v : xm) planes += (v >> m) & 1;
        C->fy_share[m] = (double)planes / S.N;
        for (int wi = 0; wi < 2; ++wi) {
          const int W = std::min(wi == 0 ? 32 : 16, S.N);  // float32, float64 tile widths
          int64_t tiles = 0;
          for (size_t t = 0; t < fm.size() / W; ++t) {
            unsigned any = 0;
            for (int p = 0; p < W; ++p) any |= fm[t * W + p];
            tiles += (any >> m) & 1;
          }
          C->fz_share[wi][m] = (double)tiles / (double)(fm.size() / W);
        }
      }
    }
    C->irr_ptr = dupload(S.irr_ptr, o, s);
    C->arm_t = dupload(S.arm_t, o, s);
    C->arm_o = dupload(S.arm_o, o, s);
    C->arm_a = dupload(S.arm_a, o, s);
    C->itp_idx = dupload(S.itp_idx, o, s);
    C->itp_w = dupload(S.itp_w, o, s);
    C->cp_target = dupload(S.cp_target, o, s);
    C->cp_of = dupload(S.cp_of, o, s);
    C->uT_ptr = dupload(S.uT_ptr, o, s);
    C->uT_node = dupload(S.uT_node, o, s);
    C->uT_row = dupload(S.uT_row, o, s);
    C->uT_w = dupload(S.uT_w, o, s);
    C->cT_ptr = dupload(S.cT_ptr, o, s);
    C->cT_node = dupload(S.cT_node, o, s);
    C->cT_slot = dupload(S.cT_slot, o, s);
    C->cT_a = dupload(S.cT_a, o, s);
    C->fT_ptr = dupload(S.fT_ptr, o, s);
    C->fT_entry = dupload(S.fT_entry, o, s);
    C->fT_target = dupload(S.fT_target, o, s);
    C->stab_a = dupload(S.stab_a, o, s);
    C->sv_ptr = dupload(S.sv_ptr, o, s);
    C->sv_idx = dupload(S.sv_idx, o, s);
    C->sv_w = dupload(S.sv_w, o, s);
    C->svT_ptr = dupload(S.svT_ptr, o, s);
    C->svT_row = dupload(S.svT_row, o, s);
    C->svT_w = dupload(S.svT_w, o, s);
    C->jumps = dalloc<double>(5 * S.T, o);
    C->fitvals = dalloc<double>(18 * S.n, o);
    C->ejump = dalloc<double>(3 * S.n, o);
    C->jbar = dalloc<double>(5 * S.T, o);
    C->fitbar = dalloc<double>(18 * S.T, o);
    C->F = dalloc<double>(4 * S.M, o);
    C->u = dalloc<double>(3 * S.M, o);
    C->p = dalloc<double>(S.M, o);
    const double c = (S.pde == KFBI_STOKES) ? 0.0 : 1.0 / (S.lam + S.mu);
    C->mixed = (C->cfg.precision == KFBI_MIXED_FP32);
    if (C->mixed) {
      C->s32.init(S.N, S.h, S.pde, S.mu, c, s, o);
      C->ru = dalloc<double>(4 * S.M, o);
      C->r32 = dalloc<float>(4 * S.M, o);
      C->r32b = dalloc<float>(4 * S.M, o);
      C->x32 = dalloc<float>(4 * S.M, o);
      C->rscal = dalloc<double>(16, o);
      C->rpart = dalloc<double>(3 * 2048, o);
    } else {
      C->s64.init(S.N, S.h, S.pde, S.mu, c, s, o);
    }
    C->s32.clock = &C->clock;
    C->s64.clock = &C->clock;
    {  // surface-stage bytes: one read of every map entry used, gathers counted per element
      const double T = (double)S.T, n = (double)S.n, nnz = (double)S.nb_idx.size();
      const double nirr = (double)S.irr_node.size(), narm = (double)S.arm_t.size();
      C->bytes_jumps = 8 * (T + 1) + nnz * (4 + 48 + 24) + T * (720 + 8 + 40) + 144 * n  // k_fit_jump
                       + n * (8 + 144 + 432 + 24);                                      // k_interp_jump
      C->bytes_correct = nirr * (8 + 8 + 8) + narm * (4 + 1 + 24 + 24);
      C->bytes_interp = 3 * n * (8 + 80 + 80 + 80 + 8);                                  // k_interp
      if (C->cfg.trace == KFBI_TRACE_AVERAGE)
        C->bytes_interp += (double)S.sv_idx.size() * (4 + 8 + 24) + 3 * n * (8 + 8 + 8 + 8) + 8 * (n + 1);
    }
    HIPCHK(hipStreamSynchronize(s));
  } catch (const DevErr& de) {
    g_create_error = de.msg;
    return KFBI_EDEVICE;
  }
  *out = C.release();
  return KFBI_OK;
}

void kfbi_destroy(kfbi_ctx* ctx) { delete ctx; }

const char* kfbi_last_error(const kfbi_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }
const char* kfbi_create_error(void) { return g_create_error.c_str(); }

kfbi_status kfbi_num_points(const kfbi_ctx* ctx, int64_t* n) {
  if (!ctx || !n) return KFBI_EINVAL;
  *n = ctx->S.n;
  return KFBI_OK;
}

kfbi_status kfbi_get_points(const kfbi_ctx* ctx, double* xyz, double* normal) {
  if (!ctx || !xyz) return KFBI_EINVAL;
  const Setup& S = ctx->S;
  for (int64_t c = 0; c < S.n; ++c)
    for (int d = 0; d < 3; ++d) {
      xyz[3 * c + d] = S.xyz[3 * S.cp_target[c] + d];
      if (normal) normal[3 * c + d] = S.nrm[3 * S.cp_target[c] + d];
    }
  return KFBI_OK;
}

kfbi_status kfbi_sizes(const kfbi_ctx* ctx, int64_t* n_crossings, int64_t* n_irregular) {
  if (!ctx) return KFBI_EINVAL;
  if (n_crossings) *n_crossings = ctx->S.T;
  if (n_irregular) *n_irregular = (int64_t)ctx->S.irr_node.size();
  return KFBI_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// pipeline
// ---------------------------------------------------------------------------------------
namespace {

// Non-finite check of an input vector: the check kernel stores a fresh tag of this check into
// pinned host memory when it meets a non-finite value; the host reads it at the call's next
// synchronisation (finish_input_check, or guarded() when the call fails), so the check costs
// no synchronisation and no copy of its own. A tag, not a cleared flag: a store of an earlier
// check that is still in flight cannot be taken for this one.
void check_finite(kfbi_ctx* C, const double* v, int64_t n) {
  C->check_tag = C->check_tag == INT32_MAX ? 1 : C->check_tag + 1;
  HIPCHK(launch_check_finite(n, v, C->hflag_dev, C->check_tag, C->s));
}
// after a synchronisation (no check kernel in flight): did the latest check see a non-finite
// value? A seen flag is consumed (tags only grow, so a later check never reuses it).
bool input_flagged(kfbi_ctx* C) {
  const bool b = C->check_tag != 0 && *C->hflag == C->check_tag;
  if (b) *C->hflag = 0;
  return b;
}
void finish_input_check(kfbi_ctx* C) {
  HIPCHK(hipStreamSynchronize(C->s));
  if (input_flagged(C)) throw std::invalid_argument("non-finite input");
}

// blocks of the refinement passes and of the correction pass that stands in for the first of them
// (3 partial sums each; 2048 measured slower)
constexpr int kRefineParts = 1024;

// right-hand side F (4 fields) from the density (and, with vol, the stored body force)
void assemble_rhs(kfbi_ctx* C, const double* phi, bool vol) {
  const Setup& S = C->S;
  hipStream_t s = C->s;
  const bool force = vol && C->has_force;
  const double* Fj = force ? C->Fj : nullptr;
  const Bat& bt = C->bt;
  const double nb = bt.nb;
  C->clock.mark(ST_JUMPS, s);
  HIPCHK(launch_fit_jump(S.T, C->nb_ptr, C->nb_idx, C->fitw, C->jmap, C->jfmap, Fj, phi, C->cp_of, C->jumps,
                         C->fitvals, s, bt));
  HIPCHK(launch_interp_jump(S.n, C->cp_target, C->fitvals, C->emap, C->efmap, Fj, C->ejump, s, bt));
  C->clock.mark(ST_CORRECT, s);
  C->bytes_extra += C->bytes_jumps * nb + C->bytes_correct * nb;
  if (!C->f_clean) {
    HIPCHK(launch_fill<double>(4 * S.M, C->F, 0.0, s, bt));
    C->bytes_extra += 32.0 * (double)S.M * nb;
  }
  const bool sparse = !(force && C->nvol);
  const int64_t nirr = (int64_t)S.irr_node.size();
  if (C->mixed && sparse) {
    // F is the corrections alone: the float32 right-hand side of the first refinement round
    // and its norm partials come from the correction pass (no dense pass over F)
    if (!C->r32_clean) {
      HIPCHK(launch_fill<float>(4 * S.M, C->r32, 0.0f, s, bt));
      C->bytes_extra += 16.0 * (double)S.M * nb;
    }
    HIPCHK(launch_correct(nirr, C->irr_node, C->irr_ptr, C->arm_t, C->arm_o, C->arm_a, C->jumps, C->F, s, C->r32,
                          S.M, C->rpart, kRefineParts, bt));
    C->r32_clean = true;
    C->r32_ready = true;
  } else {
    HIPCHK(launch_correct(nirr, C->irr_node, C->irr_ptr, C->arm_t, C->arm_o, C->arm_a, C->jumps, C->F, s, nullptr, 0,
                          nullptr, 0, bt));
    C->r32_ready = false;
  }
  C->f_clean = true;
  if (!sparse) {
    HIPCHK(launch_scatter_add(C->nvol, C->vol_idx, C->vol_val, C->F, s));
    C->bytes_extra += 24.0 * (double)C->nvol;
    C->f_clean = false;
  }
}

// float64 MAC solve of C->F into C->u, C->p (either directly or by mixed refinement)
// lean (evaluations of K phi): only the velocity is needed, and only where the interpolation
// reads it.  The mixed form then checks its first refinement round with a norms-only residual
// pass; when every right-hand side meets the tolerance there, the float64 iterate of that round
// is never stored: C->u_x32 is set and the velocity is to be read from x32 (launch_interp_x32),
// the pressure is left unset.  Otherwise the full first-round pass stores the iterate and the
// rounds go on as usual.
int mac_solve(kfbi_ctx* C, const double* F, double* u, double* p, kfbi_info* info, bool lean = false) {
  const Setup& S = C->S;
  C->u_x32 = false;
  const int64_t M = S.M;
  hipStream_t s = C->s;
  const Bat& bt = C->bt;
  const int NB = bt.nb;
  std::vector<int> its(NB, 0);
  auto sum_its = [&] {
    int t = 0;
    for (int v : its) t += v;
    return t;
  };
  // F zero outside the irregular nodes (the corrections alone): the right-hand-side transforms
  // skip the tiles without any, and the refinement reads F only in their pencils
  const bool f_sparse = F == C->F && C->f_clean;
  auto sparse_rhs = [&](auto& sv, bool on) {
    const int wi = sizeof(*sv.x) == 4 ? 0 : 1;
    sv.sp_pmask = on ? C->fmask : nullptr;
    sv.sp_xmask = on ? C->fxmask : nullptr;
    for (int m = 0; m < 3; ++m) {
      sv.sp_zread[m] = on ? C->fz_share[wi][m] : 1.0;
      sv.sp_yread[m] = on ? C->fy_share[m] : 1.0;
    }
  };
  struct SparseOff {  // no solver keeps the sparse flags past this call, exceptions included
    kfbi_ctx* C;
    ~SparseOff() {
      C->s32.sp_pmask = C->s32.sp_xmask = nullptr;
      C->s64.sp_pmask = C->s64.sp_xmask = nullptr;
    }
  } sparse_off{C};
  if (!C->mixed) {
    sparse_rhs(C->s64, f_sparse);
    int it = C->s64.solve(F, F + 3 * M, u, p, C->cfg.cg_rtol, C->cfg.cg_maxit, nullptr, &its);
    sparse_rhs(C->s64, false);
    if (it < 0) throw std::runtime_error("ENOCONV: Schur CG reached cg_maxit");
    if (info) {
      info->cg_iters += NB == 1 ? it : sum_its();
      info->refine_rounds = 0;
    }
    return it;
  }
  // mixed: float32 inner solves inside float64 residual refinement of the full system.
  // Round k: x32 = (float32 MAC solve of r32); (u, p) += x32 and r32 = F - A(u, p), formed in
  // float64 in one fused pass; stop when |r| <= cg_rtol |F| (Stokes: pressure parts taken
  // modulo constants, which the inner solve projects out).  In a batch every right-hand side
  // leaves the rounds when its own residual meets the tolerance.
  const bool stokes = S.pde == KFBI_STOKES;
  const double c = stokes ? 0.0 : 1.0 / (S.lam + S.mu);
  const double Md = (double)M;
  constexpr int NP = kRefineParts;
  Bat bref = bt;  // the refinement's launches: the right-hand sides still refining
  if (NB > 1) bref.act = C->bat_act + 2 * C->bat_cap;
  std::vector<char> live(NB, 1);
  if (NB > 1) {
    std::vector<int> ones(NB, 1);
    HIPCHK(hipMemcpyAsync(const_cast<int*>(bref.act), ones.data(), NB * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  // |F| and |r| of every right-hand side in pinned host memory (f0 read with the first residual)
  // (written by the reduction kernels through the device addresses hf0_dev, hrn_dev)
  double* hf0 = NB > 1 ? C->hpin_bat : C->hpin + 1;
  double* hrn = NB > 1 ? C->hpin_bat + NB : C->hpin;
  double* hf0_dev = NB > 1 ? C->hpin_bat_dev : C->hpin_dev + 1;
  double* hrn_dev = NB > 1 ? C->hpin_bat_dev + NB : C->hpin_dev;
  // the first inner solve is queued without a synchronisation (F = 0 gives x32 = 0 and a zero
  // residual)
  if (!(C->r32_ready && C->f_clean && F == C->F)) {
    HIPCHK(launch_refine_prep(M, F, C->r32, C->rpart, NP, s, bt));
    C->bytes_extra += 48.0 * Md * NB;
    C->r32_clean = false;
  }
  C->r32_ready = false;
  HIPCHK(launch_reduce(C->rpart, NP, 3, C->rscal, R_RESNORM0, stokes, M, s, nullptr, bt, hf0_dev));
  const double* shift = stokes ? C->rscal + 6 : nullptr;  // mean of F_p (Stokes)
  // F zero outside the irregular nodes (the corrections alone): read only in their pencils
  const uint8_t* fm = f_sparse ? C->fmask : nullptr;
  const double fbytes = 32.0 * (fm ? C->fmask_frac : 1.0);  // F bytes read per cell
  // the iterate alternates between (u, p) and the spare float64 fields (neighbour values of
  // the old iterate are read while the new one is written); in_ru[r]: where right-hand side r
  // left its final iterate
  double* cu = u;
  double* cp = p;
  std::vector<char> in_ru(NB, 0);
  int total = 0, rounds = 0, nlive = NB;
  while (nlive > 0) {
    if (rounds >= 30) throw std::runtime_error("ENOCONV: mixed refinement did not converge");
    const float* rin = (rounds == 0) ? C->r32 : C->r32b;
    std::fill(its.begin(), its.end(), 0);
    // Stokes: the pressure correction enters the residual only through its gradient, and the
    // final pressure is projected after the rounds
    sparse_rhs(C->s32, f_sparse && rounds == 0);  // the first round's right-hand side is F itself
    int it = C->s32.solve(rin, rin + 3 * M, C->x32, C->x32 + 3 * M, C->cfg.inner_rtol, C->cfg.cg_maxit, &live, &its,
                          !stokes);
    sparse_rhs(C->s32, false);
    if (it < 0) throw std::runtime_error("ENOCONV: inner float32 CG reached cg_maxit");
    total += NB == 1 ? it : sum_its();
    double* nu = (rounds == 0 || cu != u) ? u : C->ru;
    double* np = (rounds == 0 || cu != u) ? p : C->ru + 3 * M;
    C->clock.mark(ST_CG, s);
    const bool norms_only = lean && rounds == 0;
    HIPCHK(launch_refine_residual(rounds == 0, S.N, S.h, S.mu, c, cu, cp, C->x32, F, shift, nu, np, C->r32b, C->rpart,
                                  NP, s, bref, norms_only, fm));
    C->bytes_extra += ((norms_only ? 16.0 : rounds == 0 ? 64.0 : 96.0) + fbytes) * Md * nlive;
    cu = nu;
    cp = np;
    HIPCHK(launch_reduce(C->rpart, NP, 3, C->rscal, R_RESNORM, stokes, M, s, nullptr, bref, hrn_dev));
    HIPCHK(hipStreamSynchronize(s));
    ++rounds;
    for (int r = 0; r < NB; ++r) {
      if (!live[r]) continue;
      const double rn = std::sqrt(std::max(hrn[r], 0.0)), f0 = std::sqrt(std::max(hf0[r], 0.0));
      if (std::isnan(rn) || std::isnan(f0)) throw DevErr{"NaN in the refinement residual"};
      if (!(rn > C->cfg.cg_rtol * f0)) {
        live[r] = 0;
        --nlive;
        in_ru[r] = nu != u;
        if (NB > 1) HIPCHK(launch_fill<int>(1, const_cast<int*>(bref.act) + r, 0, s));
      }
    }
    if (norms_only) {
      if (nlive == 0) {  // the velocity stays in x32
        C->u_x32 = true;
        if (info) {
          info->cg_iters += total;
          info->refine_rounds = rounds;
        }
        return total;
      }
      // a right-hand side refines further: the full first-round pass stores the iterate of
      // every right-hand side of the call (and the residual of the next round)
      HIPCHK(launch_refine_residual(true, S.N, S.h, S.mu, c, u, p, C->x32, F, shift, u, p, C->r32b, C->rpart, NP, s,
                                    bt, false, fm));
      C->bytes_extra += (64.0 + fbytes) * Md * NB;
    }
  }
  for (int r = 0; r < NB; ++r)
    if (in_ru[r]) {
      HIPCHK(hipMemcpyAsync(C->s32.at(u, r), C->s32.at(C->ru, r), 3 * M * sizeof(double), hipMemcpyDeviceToDevice, s));
      HIPCHK(hipMemcpyAsync(C->s32.at(p, r), C->s32.at(C->ru + 3 * M, r), M * sizeof(double), hipMemcpyDeviceToDevice,
                            s));
      C->bytes_extra += 64.0 * Md;
    }
  if (stokes) {
    HIPCHK(launch_sum_partials<double>(M, p, C->rpart, NP, s, bt));
    HIPCHK(launch_reduce(C->rpart, NP, 1, C->rscal, R_SUM, 1, M, s, nullptr, bt));
    HIPCHK(launch_add_scalar<double>(M, p, C->rscal, 5, -1.0 / (double)M, s, bt));
    C->bytes_extra += 24.0 * Md * NB;
  }
  if (info) {
    info->cg_iters += total;
    info->refine_rounds = rounds;
  }
  return total;
}

// bytes counted by the solvers and the surface stages since the last call, into info
void take_bytes(kfbi_ctx* C, kfbi_info* info) {
  const double b = C->bytes_extra + C->s32.bytes + C->s64.bytes;
  C->bytes_extra = C->s32.bytes = C->s64.bytes = 0;
  if (info) info->model_bytes += b;
}

void eval_impl(kfbi_ctx* C, const double* phi, double* out, bool vol, kfbi_info* info) {
  const Setup& S = C->S;
  hipStream_t s = C->s;
  // stage times from events on the stream (no synchronisation between the stages)
  assemble_rhs(C, phi, vol);
  mac_solve(C, C->F, C->u, C->p, info, true);
  C->clock.mark(ST_INTERP, s);
  if (C->u_x32)
    HIPCHK(launch_interp_x32(S.n, C->itp_idx, C->itp_w, C->x32, S.N, C->ejump, out, s, C->bt));
  else
    HIPCHK(launch_interp(S.n, C->itp_idx, C->itp_w, C->u, C->ejump, out, s, C->bt));
  if (C->cfg.trace == KFBI_TRACE_AVERAGE)
    HIPCHK(launch_stab(S.n, C->sv_ptr, C->sv_idx, C->sv_w, C->stab_a, phi, out, s, C->bt));
  C->bytes_extra += C->bytes_interp * C->bt.nb;
  C->clock.mark(ST_END, s);
  HIPCHK(hipStreamSynchronize(s));
  C->clock.collect(info);
  take_bytes(C, info);
}

// Transpose of (density -> grid velocity of the double-layer interface problem), applied to
// the velocity cotangent already in C->F (F_p part zero); adds the interpolation jump term
// for the cotangent w of K phi when w != nullptr.
void transpose_from_velocity(kfbi_ctx* C, const double* w, double* out, kfbi_info* info) {
  const Setup& S = C->S;
  const int64_t M = S.M;
  hipStream_t s = C->s;
  // transpose of the MAC solve: (F_u-bar, F_p-bar) = (u', -p') with (u', p') = solve(u-bar, 0)
  mac_solve(C, C->F, C->u, C->p, info);
  C->f_clean = false;
  C->clock.mark(ST_CORRECT, s);
  HIPCHK(hipMemcpyAsync(C->F, C->u, 3 * M * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(launch_axpby<double>(M, C->F + 3 * M, -1.0, C->p, 0.0, s));
  C->bytes_extra += 72.0 * (double)M;
  // corrections^T, jump maps^T (plus the interpolation jump term), fit^T
  HIPCHK(launch_correct_T(S.T, C->cT_ptr, C->cT_node, C->cT_slot, C->cT_a, C->F, C->jbar, s));
  C->bytes_extra += C->bytes_correct;
  C->clock.mark(ST_JUMPS, s);
  HIPCHK(launch_jump_T(S.T, C->cp_of, C->jmap, C->emap, C->jbar, w, C->fitbar, s));
  HIPCHK(launch_fit_T(S.n, C->fT_ptr, C->fT_entry, C->fT_target, C->fitw, C->fitbar, out, s));
  C->bytes_extra += C->bytes_jumps;
}

void adjoint_impl(kfbi_ctx* C, const double* w, double* out, kfbi_info* info) {
  const Setup& S = C->S;
  const int64_t M = S.M;
  hipStream_t s = C->s;
  // u-bar = W^T w (F holds the solve's right-hand side (u-bar, 0))
  C->f_clean = false;
  C->clock.mark(ST_INTERP, s);
  HIPCHK(launch_fill<double>(4 * M, C->F, 0.0, s));
  HIPCHK(launch_interp_T((int64_t)S.uT_node.size(), C->uT_ptr, C->uT_node, C->uT_row, C->uT_w, w, C->F, s));
  C->bytes_extra += 32.0 * (double)M + C->bytes_interp;
  transpose_from_velocity(C, w, out, info);
  if (C->cfg.trace == KFBI_TRACE_AVERAGE) {
    C->clock.mark(ST_INTERP, s);
    HIPCHK(launch_stab_T(S.n, C->svT_ptr, C->svT_row, C->svT_w, C->stab_a, w, out, s));
  }
  C->clock.mark(ST_END, s);
  HIPCHK(hipStreamSynchronize(s));
  C->clock.collect(info);
  take_bytes(C, info);
}

template <typename F>
kfbi_status guarded(kfbi_ctx* C, F&& f) {
  if (!C) return KFBI_EINVAL;
  auto bad_input = [&]() -> bool {  // a failure caused by a non-finite input reports EINVAL
    (void)hipStreamSynchronize(C->s);
    return input_flagged(C);
  };
  C->clock.used = 0;
  C->bytes_extra = C->s32.bytes = C->s64.bytes = 0;
  try {
    f();
    return KFBI_OK;
  } catch (const DevErr& e) {
    C->err = e.msg;
    if (bad_input()) {
      C->err = "non-finite input";
      return KFBI_EINVAL;
    }
    return KFBI_EDEVICE;
  } catch (const std::invalid_argument& e) {
    C->err = e.what();
    return KFBI_EINVAL;
  } catch (const std::runtime_error& e) {
    C->err = e.what();
    if (bad_input()) {
      C->err = "non-finite input";
      return KFBI_EINVAL;
    }
    return std::string(e.what()).rfind("ENOCONV", 0) == 0 ? KFBI_ENOCONV : KFBI_EDEVICE;
  } catch (const std::bad_alloc&) {
    C->err = "host allocation failed";
    return KFBI_ENOMEM;
  }
}

// The per-call work buffers of an evaluation (everything kfbi_eval writes besides its output):
// swapped for buffers carved from the no-alloc scratch for one call, then restored.
struct WorkSet {
  double *jumps, *fitvals, *ejump, *F, *u, *p, *ru, *rscal, *rpart;
  float *r32, *r32b, *x32;
  SolverPtrs<float> s32;
  SolverPtrs<double> s64;
  bool f_clean, r32_clean, r32_ready;
  int prof32, prof64;
};

WorkSet get_work(const kfbi_ctx* C) {
  return {C->jumps, C->fitvals, C->ejump, C->F, C->u, C->p, C->ru, C->rscal, C->rpart, C->r32, C->r32b, C->x32,
          C->s32.ptrs(), C->s64.ptrs(), C->f_clean, C->r32_clean, C->r32_ready,
          C->s32.prof_kind, C->s64.prof_kind};
}

void set_work(kfbi_ctx* C, const WorkSet& w) {
  C->jumps = w.jumps, C->fitvals = w.fitvals, C->ejump = w.ejump, C->F = w.F, C->u = w.u, C->p = w.p;
  C->ru = w.ru, C->rscal = w.rscal, C->rpart = w.rpart, C->r32 = w.r32, C->r32b = w.r32b, C->x32 = w.x32;
  if (C->mixed)
    C->s32.set(w.s32);
  else
    C->s64.set(w.s64);
  C->f_clean = w.f_clean, C->r32_clean = w.r32_clean, C->r32_ready = w.r32_ready;
  C->s32.prof_kind = w.prof32, C->s64.prof_kind = w.prof64;
}

// the work buffers of one evaluation carved from an arena (sizes as in kfbi_create); the scratch
// keeps whatever the last call left, so every buffer that is read before it is written starts
// dirty (dense clears of F and of the float32 right-hand side) and profiling is off
WorkSet carve_work(const kfbi_ctx* C, Arena& a) {
  const Setup& S = C->S;
  WorkSet w = get_work(C);
  w.jumps = a.take<double>(5 * S.T);
  w.fitvals = a.take<double>(18 * S.n);
  w.ejump = a.take<double>(3 * S.n);
  w.F = a.take<double>(4 * S.M);
  w.u = a.take<double>(3 * S.M);
  w.p = a.take<double>(S.M);
  if (C->mixed) {
    w.ru = a.take<double>(4 * S.M);
    w.r32 = a.take<float>(4 * S.M);
    w.r32b = a.take<float>(4 * S.M);
    w.x32 = a.take<float>(4 * S.M);
    w.rscal = a.take<double>(16);
    w.rpart = a.take<double>(3 * 2048);
    w.s32 = C->s32.carve(a);
  } else {
    w.s64 = C->s64.carve(a);
  }
  w.f_clean = w.r32_clean = w.r32_ready = false;
  w.prof32 = w.prof64 = -1;
  return w;
}

// bytes of the no-alloc scratch an evaluation on this context needs
size_t noalloc_bytes(const kfbi_ctx* C) {
  Arena a;
  (void)carve_work(C, a);
  return a.used;
}

// Work arenas of a batch of nrhs right-hand sides (each carved like the context's own work
// buffers, bat_A bytes apart), their flags and the pinned host slots of their scalars.
void ensure_batch(kfbi_ctx* C, int nrhs) {
  if (nrhs <= C->bat_cap) return;
  const int64_t A = ((int64_t)noalloc_bytes(C) + 4095) / 4096 * 4096;
  dfree(C->bat_base, C->owned);
  dfree(C->bat_act, C->owned);
  C->bat_base = nullptr;
  C->bat_act = nullptr;
  C->bat_cap = C->bat_clean = 0;
  void* base = nullptr;
  if (hipMalloc(&base, (size_t)A * nrhs) != hipSuccess) {
    (void)hipGetLastError();
    throw std::bad_alloc();
  }
  C->owned.push_back(base);
  C->bat_base = static_cast<char*>(base);
  C->bat_A = A;
  C->bat_act = dalloc<int>(3 * nrhs, C->owned);
  if (C->hpin_bat) (void)hipHostFree(C->hpin_bat);
  C->hpin_bat = C->hpin_bat_dev = nullptr;
  HIPCHK(hipHostMalloc((void**)&C->hpin_bat, 2 * nrhs * sizeof(double), hipHostMallocDefault));
  HIPCHK(hipHostGetDevicePointer((void**)&C->hpin_bat_dev, C->hpin_bat, 0));
  auto grow_rr = [&](auto& sv) {
    if (sv.host_rr) (void)hipHostFree(sv.host_rr);
    sv.host_rr = nullptr;
    sv.host_rr_dev = nullptr;
    HIPCHK(hipHostMalloc((void**)&sv.host_rr, 16 * nrhs * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipHostGetDevicePointer((void**)&sv.host_rr_dev, sv.host_rr, 0));
    sv.rr_cap = nrhs;
  };
  if (C->mixed)
    grow_rr(C->s32);
  else
    grow_rr(C->s64);
  C->bat_cap = nrhs;
}

// transpose of density -> probe values of the unified interface solve (the affine body-force
// part drops out), into phi_bar
void probe_adjoint_impl(kfbi_ctx* C, const double* vals_bar, double* phi_bar, kfbi_info* info) {
  hipStream_t s = C->s;
  C->f_clean = false;
  C->clock.mark(ST_INTERP, s);
  HIPCHK(launch_fill<double>(4 * C->S.M, C->F, 0.0, s));
  HIPCHK(launch_interp_T(C->nprobe_nodes, C->prT_ptr, C->prT_node, C->prT_row, C->prT_w, vals_bar, C->F, s));
  C->bytes_extra += 32.0 * (double)C->S.M;
  transpose_from_velocity(C, nullptr, phi_bar, info);
  C->clock.mark(ST_END, s);
  HIPCHK(hipStreamSynchronize(s));
  C->clock.collect(info);
  take_bytes(C, info);
}

// GMRES dot product into a device slot (float64, deterministic)
void dev_dot(kfbi_ctx* C, const double* a, const double* b, int64_t n, double* slot) {
  HIPCHK(launch_dot_partials<double>(n, a, b, C->rpart, 64, C->s));
  HIPCHK(launch_reduce(C->rpart, 64, 1, C->rscal, R_SUM, 0, n, C->s, slot));
}

}  // namespace

// GMRES device helpers (small kernels)
__global__ void k_axpy_dev(int64_t n, double* y, const double* x, const double* a, double sign) {
  const double av = sign * (*a);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += av * x[i];
}
__global__ void k_scale_inv_norm(int64_t n, double* y, const double* nsq, double* hout) {
  const double nv = sqrt(*nsq);
  if (blockIdx.x == 0 && threadIdx.x == 0) *hout = nv;
  const double f = (nv > 0) ? 1.0 / nv : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] *= f;
}

namespace {

// unrestarted GMRES (modified Gram-Schmidt, Givens rotations) on K phi = rhs, zero guess
void adjoint_impl(kfbi_ctx* C, const double* w, double* out, kfbi_info* info);

// unrestarted GMRES (modified Gram-Schmidt, Givens rotations) on K x = rhs (or K^T x = rhs)
int gmres(kfbi_ctx* C, const double* rhs, double* phi, double tol, int maxit, double* relres, kfbi_info* info,
          bool transpose = false) {
  const Setup& S = C->S;
  const int64_t n3 = 3 * S.n;
  hipStream_t s = C->s;
  if (C->gm_max < maxit) {  // Krylov basis and Hessenberg columns, regrown (old buffers freed)
    dfree(C->V, C->owned);
    dfree(C->H, C->owned);
    C->V = C->H = nullptr;
    C->gm_max = 0;
    C->V = dalloc<double>((size_t)(maxit + 1) * n3, C->owned);
    C->H = dalloc<double>((size_t)(maxit + 2) * (maxit + 1) + 16, C->owned);
    C->gm_max = maxit;
  }
  if (!C->rpart) C->rpart = dalloc<double>(3 * 2048, C->owned);
  if (!C->rscal) C->rscal = dalloc<double>(16, C->owned);
  const int LD = maxit + 2;  // column stride of H
  double* sc = C->rscal;  // sc[5] = norm^2, sc[6] = norm
  HIPCHK(hipMemcpyAsync(C->V, rhs, n3 * sizeof(double), hipMemcpyDeviceToDevice, s));
  dev_dot(C, C->V, C->V, n3, sc + 5);
  double beta2 = 0;
  HIPCHK(hipMemcpyAsync(&beta2, sc + 5, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double beta = std::sqrt(beta2);
  HIPCHK(launch_fill<double>(n3, phi, 0.0, s));
  if (beta == 0) {
    *relres = 0;
    return 0;
  }
  hipLaunchKernelGGL(k_scale_inv_norm, dim3(64), dim3(256), 0, s, n3, C->V, sc + 5, sc + 6);
  std::vector<double> Hh((size_t)LD * (maxit + 1), 0.0), cs(maxit + 1), sn(maxit + 1), g(maxit + 2, 0.0);
  g[0] = beta;
  int k = 0;
  double res = 1.0;
  for (k = 0; k < maxit; ++k) {
    double* vk = C->V + (size_t)k * n3;
    double* w = C->V + (size_t)(k + 1) * n3;
    if (transpose)
      adjoint_impl(C, vk, w, info);
    else
      eval_impl(C, vk, w, false, info);
    double* Hc = C->H + (size_t)k * LD;
    for (int i = 0; i <= k; ++i) {
      dev_dot(C, C->V + (size_t)i * n3, w, n3, Hc + i);
      hipLaunchKernelGGL(k_axpy_dev, dim3(64), dim3(256), 0, s, n3, w, C->V + (size_t)i * n3, Hc + i, -1.0);
    }
    dev_dot(C, w, w, n3, sc + 5);
    hipLaunchKernelGGL(k_scale_inv_norm, dim3(64), dim3(256), 0, s, n3, w, sc + 5, Hc + k + 1);
    HIPCHK(hipGetLastError());
    std::vector<double> col(k + 2);
    HIPCHK(hipMemcpyAsync(col.data(), Hc, (k + 2) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < k; ++i) {
      double a = col[i], b = col[i + 1];
      col[i] = cs[i] * a + sn[i] * b;
      col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    double r = std::hypot(col[k], col[k + 1]);
    cs[k] = col[k] / r;
    sn[k] = col[k + 1] / r;
    col[k] = r;
    col[k + 1] = 0;
    for (int i = 0; i <= k; ++i) Hh[(size_t)k * LD + i] = col[i];
    g[k + 1] = -sn[k] * g[k];
    g[k] = cs[k] * g[k];
    res = std::fabs(g[k + 1]) / beta;
    if (res < tol) {
      ++k;
      break;
    }
  }
  const int m = std::min(k, maxit);
  std::vector<double> y(m);
  for (int i = m - 1; i >= 0; --i) {
    double acc = g[i];
    for (int j = i + 1; j < m; ++j) acc -= Hh[(size_t)j * LD + i] * y[j];
    y[i] = acc / Hh[(size_t)i * LD + i];
  }
  for (int i = 0; i < m; ++i)
    HIPCHK(launch_axpby<double>(n3, phi, y[i], C->V + (size_t)i * n3, 1.0, s));
  HIPCHK(hipStreamSynchronize(s));
  *relres = res;
  if (info) {
    info->gmres_iters = m;
    info->final_rel_residual = res;
  }
  if (res >= tol) throw std::runtime_error("ENOCONV: GMRES reached gmres_maxit");
  return m;
}

void set_volume_force(kfbi_ctx* C, kfbi_vec_fn f, void* user) {
  Setup& S = C->S;
  const int N = S.N;
  hipStream_t s = C->s;
  // nodes of T^1..T^3 inside Omega (interior faces only)
  std::vector<double> xyz;
  std::vector<int64_t> idx;
  for (int m = 0; m < 3; ++m)
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j)
        for (int k = 0; k < N; ++k) {
          const int id[3] = {i, j, k};
          if (id[m] == 0) continue;
          const int64_t l = ((int64_t)i * N + j) * N + k;
          if (!S.side[m][l]) continue;
          for (int d = 0; d < 3; ++d) xyz.push_back(d == m ? S.lo + id[d] * S.h : S.lo + (id[d] + 0.5) * S.h);
          idx.push_back((int64_t)m * S.M + l);
        }
  const int64_t nv = (int64_t)idx.size();
  std::vector<double> fv(3 * nv), val(nv);
  if (nv) f(xyz.data(), nv, fv.data(), user);
  for (int64_t r = 0; r < nv; ++r) {
    const int m = (int)(idx[r] / S.M);
    val[r] = fv[3 * r + m];
    if (!std::isfinite(val[r])) throw std::invalid_argument("non-finite body force");
  }
  std::vector<double> Fj(3 * S.T);
  f(S.xyz.data(), S.T, Fj.data(), user);
  for (double v : Fj)
    if (!std::isfinite(v)) throw std::invalid_argument("non-finite body force");
  C->has_force = false;
  if (!C->Fj) C->Fj = dalloc<double>(3 * S.T, C->owned);
  HIPCHK(hipMemcpyAsync(C->Fj, Fj.data(), Fj.size() * sizeof(double), hipMemcpyHostToDevice, s));
  if (C->vol_cap < nv || !C->vol_idx) {
    dfree(C->vol_idx, C->owned);
    dfree(C->vol_val, C->owned);
    C->vol_idx = nullptr;
    C->vol_val = nullptr;
    C->vol_cap = 0;
    C->vol_idx = dalloc<int64_t>(std::max<int64_t>(nv, 1), C->owned);
    C->vol_val = dalloc<double>(std::max<int64_t>(nv, 1), C->owned);
    C->vol_cap = std::max<int64_t>(nv, 1);
  }
  C->nvol = nv;
  if (nv) {
    HIPCHK(hipMemcpyAsync(C->vol_idx, idx.data(), nv * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(C->vol_val, val.data(), nv * sizeof(double), hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  C->has_force = true;
}

}  // namespace

extern "C" {

kfbi_status kfbi_eval(kfbi_ctx* C, const double* phi, double* out, kfbi_info* info) {
  if (!C || !phi || !out) return KFBI_EINVAL;
  if (info) std::memset(info, 0, sizeof(*info));
  return guarded(C, [&] {
    check_finite(C, phi, 3 * C->S.n);
    eval_impl(C, phi, out, false, info);
    finish_input_check(C);
  });
}

kfbi_status kfbi_eval_noalloc(kfbi_ctx* C, const double* phi, double* out, kfbi_info* info) {
  if (!C || !phi || !out) return KFBI_EINVAL;
  if (info) std::memset(info, 0, sizeof(*info));
  const size_t need = noalloc_bytes(C);
  if (need > (size_t)KFBI_NOALLOC_MAX_BYTES) {
    C->err = "kfbi_eval_noalloc: this context needs " + std::to_string(need) + " bytes of scratch, more than " +
             "KFBI_NOALLOC_MAX_BYTES = " + std::to_string((size_t)KFBI_NOALLOC_MAX_BYTES);
    return KFBI_EINVAL;
  }
  return guarded(C, [&] {
    char* base = static_cast<char*>(scratch_address(C->dev));
    if (!base) throw DevErr{"no device address of the no-alloc scratch"};
    Arena a{base, (size_t)KFBI_NOALLOC_MAX_BYTES, 0};
    const WorkSet own = get_work(C);
    set_work(C, carve_work(C, a));
    struct Restore {
      kfbi_ctx* C;
      const WorkSet& w;
      ~Restore() { set_work(C, w); }
    } restore{C, own};
    check_finite(C, phi, 3 * C->S.n);
    eval_impl(C, phi, out, false, info);
    finish_input_check(C);
  });
}

kfbi_status kfbi_eval_batch(kfbi_ctx* C, int32_t nrhs, const double* phi, double* out, kfbi_info* info) {
  if (!C || !phi || !out || nrhs < 1 || nrhs > KFBI_BATCH_MAX) return KFBI_EINVAL;
  if (info) std::memset(info, 0, sizeof(*info));
  return guarded(C, [&] {
    const int64_t n3 = 3 * C->S.n;
    check_finite(C, phi, nrhs * n3);
    ensure_batch(C, nrhs);
    const bool clean = nrhs <= C->bat_clean;
    const int clean_before = C->bat_clean;
    C->bat_clean = 0;
    const WorkSet own = get_work(C);
    Arena a{C->bat_base, (size_t)C->bat_A, 0};
    WorkSet w = carve_work(C, a);
    w.f_clean = w.r32_clean = clean;
    w.prof32 = own.prof32;
    w.prof64 = own.prof64;
    set_work(C, w);
    const Bat bt{C->bat_A, n3, nullptr, nrhs};
    auto attach = [&](auto& sv) {
      sv.bt = sv.cur = bt;
      sv.act_live = C->bat_act;
      sv.act_cg = C->bat_act + C->bat_cap;
    };
    C->bt = bt;
    attach(C->s32);
    attach(C->s64);
    struct Restore {
      kfbi_ctx* C;
      const WorkSet& w;
      ~Restore() {
        set_work(C, w);
        C->bt = C->s32.bt = C->s32.cur = C->s64.bt = C->s64.cur = Bat();
        C->s32.act_live = C->s32.act_cg = C->s64.act_live = C->s64.act_cg = nullptr;
      }
    } restore{C, own};
    eval_impl(C, phi, out, false, info);
    finish_input_check(C);
    C->bat_clean = std::max(clean_before, (int)nrhs);
  });
}

kfbi_status kfbi_eval_adjoint(kfbi_ctx* C, const double* w, double* out, kfbi_info* info) {
  if (!C || !w || !out) return KFBI_EINVAL;
  if (info) std::memset(info, 0, sizeof(*info));
  return guarded(C, [&] {
    check_finite(C, w, 3 * C->S.n);
    adjoint_impl(C, w, out, info);
    finish_input_check(C);
  });
}

kfbi_status kfbi_solve_bvp(kfbi_ctx* C, const double* g, kfbi_vec_fn f, void* user, double* phi, double* u_ext,
                           double* p_ext, kfbi_info* info) {
  if (!C || !g || !phi) return KFBI_EINVAL;
  if (info) std::memset(info, 0, sizeof(*info));
  return guarded(C, [&] {
    const Setup& S = C->S;
    const int64_t n3 = 3 * S.n;
    check_finite(C, g, n3);
    finish_input_check(C);
    if (!C->gtmp) C->gtmp = dalloc<double>(n3, C->owned);
    if (f) {
      set_volume_force(C, f, user);
      // b = trace of the volume problem (phi = 0)
      HIPCHK(launch_fill<double>(n3, phi, 0.0, C->s));
      eval_impl(C, phi, C->gtmp, true, info);
      HIPCHK(launch_axpby<double>(n3, C->gtmp, 1.0, g, -1.0, C->s));  // g - b
    } else {
      HIPCHK(hipMemcpyAsync(C->gtmp, g, n3 * sizeof(double), hipMemcpyDeviceToDevice, C->s));
    }
    double rr = 0;
    gmres(C, C->gtmp, phi, C->cfg.gmres_rtol, C->cfg.gmres_maxit, &rr, info);
    if (u_ext || p_ext) {
      assemble_rhs(C, phi, f != nullptr);
      mac_solve(C, C->F, C->u, C->p, info);
      if (u_ext) HIPCHK(launch_export_u(S.N, C->u, u_ext, C->s));
      if (p_ext) HIPCHK(hipMemcpyAsync(p_ext, C->p, S.M * sizeof(double), hipMemcpyDeviceToDevice, C->s));
      C->clock.mark(ST_END, C->s);
      HIPCHK(hipStreamSynchronize(C->s));
      C->clock.collect(info);
      take_bytes(C, info);
    }
  });
}

kfbi_status kfbi_interface_solve(kfbi_ctx* C, const double* phi, int32_t use_force, double* u_ext, double* p_ext,
                                 kfbi_info* info) {
  if (!C || !phi) return KFBI_EINVAL;
  if (info) std::memset(info, 0, sizeof(*info));
  return guarded(C, [&] {
    const Setup& S = C->S;
    check_finite(C, phi, 3 * S.n);
    assemble_rhs(C, phi, use_force != 0);
    mac_solve(C, C->F, C->u, C->p, info);
    if (u_ext) HIPCHK(launch_export_u(S.N, C->u, u_ext, C->s));
    if (p_ext) HIPCHK(hipMemcpyAsync(p_ext, C->p, S.M * sizeof(double), hipMemcpyDeviceToDevice, C->s));
    C->clock.mark(ST_END, C->s);
    finish_input_check(C);
    C->clock.collect(info);
    take_bytes(C, info);
  });
}

kfbi_status kfbi_profile_pass(kfbi_ctx* C, int32_t kind, int32_t axis, int32_t enable, int64_t* launches,
                              double* total_ms, double* bytes_per_launch) {
  if (!C || kind < 0 || kind > KFBI_K_YINV || axis < -1 || axis > 2) return KFBI_EINVAL;
  return guarded(C, [&] {
    auto go = [&](auto& sv) {
      if (launches) *launches = sv.prof_launches;
      if (total_ms) *total_ms = sv.prof_ms;
      if (bytes_per_launch) *bytes_per_launch = sv.kernel_bytes(kind);
      sv.prof_kind = enable ? kind : -1;
      sv.prof_axis = enable ? axis : -1;
      sv.prof_launches = 0;
      sv.prof_ms = 0;
    };
    if (C->mixed)
      go(C->s32);
    else
      go(C->s64);
  });
}

kfbi_status kfbi_time_pass(kfbi_ctx* C, int32_t kind, int32_t axis, int32_t reps, double* avg_ms, double* bytes) {
  if (!C || !avg_ms || kind < 0 || kind > KFBI_K_GEMM_X || axis < 0 || axis > 2 || reps <= 0) return KFBI_EINVAL;
  return guarded(C, [&] {
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto run = [&](auto& sv) {
      using T = std::remove_reference_t<decltype(*sv.A)>;
      if (kind == KFBI_K_GEMM_X) sv.ensure_gemm(C->owned);
      for (T* f : {sv.A, sv.B, sv.A1, sv.B2, sv.B3, sv.r, sv.d, sv.q, sv.x})
        HIPCHK(launch_fill<T>(sv.M, f, T(1), C->s));
      HIPCHK(hipMemsetAsync(sv.scal, 0, 16 * sizeof(double), C->s));
      auto once = [&] {
        switch (kind) {
          case KFBI_K_XMID: sv.xmid(); break;
          case KFBI_K_ZFWD: sv.zfwd(); break;
          case KFBI_K_ZINV: sv.zinv(); break;
          case KFBI_K_YFWD: sv.yfwd(); break;
          case KFBI_K_YINV: sv.yinv(); break;
          case KFBI_K_GEMM_X:
            if constexpr (sizeof(T) == 4) HIPCHK(launch_gemm_dct2_x(sv.N, sv.A, sv.B, sv.gemm_cf, C->s));
            break;
          default: sv.pass(kind, axis, sv.A, sv.B);
        }
      };
      once();  // warm-up
      HIPCHK(hipEventRecord(e0, C->s));
      for (int r = 0; r < reps; ++r) once();
      HIPCHK(hipEventRecord(e1, C->s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      *avg_ms = ms / reps;
      if (bytes) *bytes = sv.kernel_bytes(kind);
    };
    if (C->mixed)
      run(C->s32);
    else
      run(C->s64);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  });
}

kfbi_status kfbi_apply_pass(kfbi_ctx* C, int32_t kind, int32_t axis, const double* in, double* out) {
  if (!C || !in || !out || kind < 0 || (kind > 4 && kind != KFBI_K_GEMM_X) || axis < 0 || axis > 2)
    return KFBI_EINVAL;
  if (kind == KFBI_K_GEMM_X && axis != 0) return KFBI_EINVAL;
  return guarded(C, [&] {
    auto run = [&](auto& sv) {
      using T = std::remove_reference_t<decltype(*sv.A)>;
      if (kind == KFBI_K_GEMM_X) sv.ensure_gemm(C->owned);
      HIPCHK((launch_convert<double, T>(sv.M, in, sv.A, C->s)));
      if (kind == KFBI_K_GEMM_X) {
        if constexpr (sizeof(T) == 4) HIPCHK(launch_gemm_dct2_x(sv.N, sv.A, sv.B, sv.gemm_cf, C->s));
      } else {
        HIPCHK(launch_pass<T>(sv.N, kind, axis, sv.A, sv.B, false, sv.tb, C->s));
      }
      HIPCHK((launch_convert<T, double>(sv.M, sv.B, out, C->s)));
      HIPCHK(hipStreamSynchronize(C->s));
    };
    if (C->mixed)
      run(C->s32);
    else
      run(C->s64);
  });
}

}  // extern "C"

template <typename V>
static int64_t copy_out(const V& v, void* out) {
  if (out) std::memcpy(out, v.data(), v.size() * sizeof(v[0]));
  return (int64_t)v.size();
}

extern "C" {

// ---------------------------------------------------------------------------------------
// host-only plan (setup without a device), used to inspect the geometry and maps
// ---------------------------------------------------------------------------------------
kfbi_status kfbi_plan_create(const kfbi_config* cfg, kfbi_plan** out) {
  if (!out) return KFBI_EINVAL;
  *out = nullptr;
  if (const char* v = validate(cfg)) {
    g_create_error = v;
    return KFBI_EINVAL;
  }
  std::unique_ptr<kfbi_plan> P(new kfbi_plan());
  P->cfg = normalized(cfg);
  std::string e;
  try {
    e = build_setup(P->cfg, P->S);
  } catch (const std::exception& ex) {
    e = std::string("setup failed: ") + ex.what();
  }
  if (!e.empty()) {
    g_create_error = e;
    return status_of_setup(e);
  }
  *out = P.release();
  return KFBI_OK;
}

void kfbi_plan_destroy(kfbi_plan* p) { delete p; }

int64_t kfbi_plan_get(const kfbi_plan* p, const char* name, void* out) {
  if (!p || !name) return -1;
  const Setup& S = p->S;
  std::string n(name);
  if (n == "xyz") return copy_out(S.xyz, out);
  if (n == "normal") return copy_out(S.nrm, out);
  if (n == "t1") return copy_out(S.t1, out);
  if (n == "t2") return copy_out(S.t2, out);
  if (n == "kappa") return copy_out(S.kap, out);
  if (n == "fam") return copy_out(S.fam, out);
  if (n == "line1") return copy_out(S.l1, out);
  if (n == "line2") return copy_out(S.l2, out);
  if (n == "cp_target") return copy_out(S.cp_target, out);
  if (n == "nb_ptr") return copy_out(S.nb_ptr, out);
  if (n == "nb_idx") return copy_out(S.nb_idx, out);
  if (n == "fitw") return copy_out(S.fitw, out);
  if (n == "jmap") return copy_out(S.jmap, out);
  if (n == "jfmap") return copy_out(S.jfmap, out);
  if (n == "emap") return copy_out(S.emap, out);
  if (n == "stab_a") return copy_out(S.stab_a, out);
  if (n == "sv_ptr") return copy_out(S.sv_ptr, out);
  if (n == "sv_idx") return copy_out(S.sv_idx, out);
  if (n == "sv_w") return copy_out(S.sv_w, out);
  if (n == "irr_node") return copy_out(S.irr_node, out);
  if (n == "irr_ptr") return copy_out(S.irr_ptr, out);
  if (n == "arm_t") return copy_out(S.arm_t, out);
  if (n == "arm_o") return copy_out(S.arm_o, out);
  if (n == "arm_a") return copy_out(S.arm_a, out);
  if (n == "itp_idx") return copy_out(S.itp_idx, out);
  if (n == "itp_w") return copy_out(S.itp_w, out);
  if (n == "side0") return copy_out(S.side[0], out);
  if (n == "side1") return copy_out(S.side[1], out);
  if (n == "side2") return copy_out(S.side[2], out);
  if (n == "sidep") return copy_out(S.side[3], out);
  return -1;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// interior probes and the adjoint solves used by the autograd layer
// ---------------------------------------------------------------------------------------
extern "C" {

kfbi_status kfbi_set_probes(kfbi_ctx* C, const double* xyz, int64_t m) {
  if (!C || (!xyz && m > 0) || m < 0) return KFBI_EINVAL;
  return guarded(C, [&] {
    const Setup& S = C->S;
    const int N = S.N;
    std::vector<int64_t> idx(m * 24);
    std::vector<double> w(m * 24);
    for (int64_t i = 0; i < m; ++i)
      for (int c = 0; c < 3; ++c) {
        int base[3];
        double t[3];
        for (int d = 0; d < 3; ++d) {
          const double off = (d == c) ? 0.0 : 0.5;
          const double u = (xyz[3 * i + d] - S.lo) / S.h - off;
          if (!std::isfinite(u)) throw std::invalid_argument("non-finite probe");
          base[d] = (int)std::floor(u);
          t[d] = u - base[d];
          const int lo_ok = (d == c) ? 1 : 0;
          if (base[d] < lo_ok || base[d] + 1 > N - 1) throw std::invalid_argument("probe outside the interior nodes");
        }
        for (int k = 0; k < 8; ++k) {
          int a[3];
          double wt = 1.0;
          for (int d = 0; d < 3; ++d) {
            const int bit = (k >> (2 - d)) & 1;
            a[d] = base[d] + bit;
            wt *= bit ? t[d] : 1.0 - t[d];
          }
          idx[(i * 3 + c) * 8 + k] = (int64_t)c * S.M + ((int64_t)a[0] * N + a[1]) * N + a[2];
          w[(i * 3 + c) * 8 + k] = wt;
        }
      }
    // transpose: CSR over distinct grid nodes
    std::vector<std::tuple<int64_t, int32_t, double>> ent;
    ent.reserve(m * 24);
    for (int64_t r = 0; r < 3 * m; ++r)
      for (int k = 0; k < 8; ++k) ent.emplace_back(idx[r * 8 + k], (int32_t)r, w[r * 8 + k]);
    std::sort(ent.begin(), ent.end());
    std::vector<int64_t> ptr(1, 0), node;
    std::vector<int32_t> row;
    std::vector<double> tw;
    for (size_t e = 0; e < ent.size(); ++e) {
      if (e == 0 || std::get<0>(ent[e]) != std::get<0>(ent[e - 1])) {
        if (e > 0) ptr.push_back((int64_t)e);
        node.push_back(std::get<0>(ent[e]));
      }
      row.push_back(std::get<1>(ent[e]));
      tw.push_back(std::get<2>(ent[e]));
    }
    ptr.push_back((int64_t)ent.size());
    auto& o = C->owned;
    C->pr_idx = dupload(idx, o, C->s);
    C->pr_w = dupload(w, o, C->s);
    C->prT_ptr = dupload(ptr, o, C->s);
    C->prT_node = dupload(node, o, C->s);
    C->prT_row = dupload(row, o, C->s);
    C->prT_w = dupload(tw, o, C->s);
    C->nprobe = m;
    C->nprobe_nodes = (int64_t)node.size();
    HIPCHK(hipStreamSynchronize(C->s));
  });
}

kfbi_status kfbi_probe(kfbi_ctx* C, const double* phi, int32_t use_force, double* vals, kfbi_info* info) {
  if (!C || !phi || !vals) return KFBI_EINVAL;
  if (info) std::memset(info, 0, sizeof(*info));
  if (C->nprobe == 0) {
    C->err = "no probes set";
    return KFBI_EINVAL;
  }
  return guarded(C, [&] {
    check_finite(C, phi, 3 * C->S.n);
    assemble_rhs(C, phi, use_force != 0);
    mac_solve(C, C->F, C->u, C->p, info);
    // trilinear interpolation: 8 weights per (probe, component)
    C->clock.mark(ST_INTERP, C->s);
    HIPCHK(launch_interp8(C->nprobe, C->pr_idx, C->pr_w, C->u, vals, C->s));
    C->clock.mark(ST_END, C->s);
    finish_input_check(C);
    C->clock.collect(info);
    take_bytes(C, info);
  });
}

kfbi_status kfbi_probe_adjoint(kfbi_ctx* C, const double* vals_bar, double* phi_bar, kfbi_info* info) {
  if (!C || !vals_bar || !phi_bar) return KFBI_EINVAL;
  if (info) std::memset(info, 0, sizeof(*info));
  if (C->nprobe == 0) {
    C->err = "no probes set";
    return KFBI_EINVAL;
  }
  return guarded(C, [&] {
    check_finite(C, vals_bar, 3 * C->nprobe);
    probe_adjoint_impl(C, vals_bar, phi_bar, info);
    finish_input_check(C);
  });
}

kfbi_status kfbi_solve_adjoint(kfbi_ctx* C, const double* rhs, double* y, kfbi_info* info) {
  if (!C || !rhs || !y) return KFBI_EINVAL;
  if (info) std::memset(info, 0, sizeof(*info));
  return guarded(C, [&] {
    const int64_t n3 = 3 * C->S.n;
    check_finite(C, rhs, n3);
    finish_input_check(C);
    if (!C->gtmp) C->gtmp = dalloc<double>(n3, C->owned);
    HIPCHK(hipMemcpyAsync(C->gtmp, rhs, n3 * sizeof(double), hipMemcpyDeviceToDevice, C->s));
    double rr = 0;
    gmres(C, C->gtmp, y, C->cfg.gmres_rtol, C->cfg.gmres_maxit, &rr, info, true);
  });
}

kfbi_status kfbi_solve_bvp_adjoint(kfbi_ctx* C, const double* vals_bar, double* g_bar, double* phi_bar,
                                   kfbi_info* info) {
  if (!C || !vals_bar || (!g_bar && !phi_bar)) return KFBI_EINVAL;
  if (info) std::memset(info, 0, sizeof(*info));
  if (C->nprobe == 0) {
    C->err = "no probes set";
    return KFBI_EINVAL;
  }
  return guarded(C, [&] {
    const int64_t n3 = 3 * C->S.n;
    check_finite(C, vals_bar, 3 * C->nprobe);
    finish_input_check(C);
    // phi-bar = P^T v-bar (probe values as a function of the density), then g-bar = K^{-T} phi-bar
    double* pb = phi_bar;
    if (!pb) {
      if (!C->pbar) C->pbar = dalloc<double>(n3, C->owned);
      pb = C->pbar;
    }
    probe_adjoint_impl(C, vals_bar, pb, info);
    HIPCHK(hipStreamSynchronize(C->s));
    if (g_bar) {
      if (!C->gtmp) C->gtmp = dalloc<double>(n3, C->owned);
      HIPCHK(hipMemcpyAsync(C->gtmp, pb, n3 * sizeof(double), hipMemcpyDeviceToDevice, C->s));
      double rr = 0;
      gmres(C, C->gtmp, g_bar, C->cfg.gmres_rtol, C->cfg.gmres_maxit, &rr, info, true);
    }
  });
}

}  // extern "C"
