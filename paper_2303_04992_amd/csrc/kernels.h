// Device kernels of the KFBI operator evaluation (launch wrappers).  All wrappers enqueue
// on the given stream and return hipSuccess or the launch error.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace kfbi {

template <typename T>
struct SpecTab;  // device tables of one precision (defined in kernels.hip)

// Several right-hand sides in one launch (lockstep batches): blockIdx.z is the right-hand side
// r < nb; every work-buffer pointer a kernel receives is that of right-hand side 0, and the one
// of right-hand side r lies r * A bytes further (each right-hand side owns one arena of A bytes,
// carved identically); caller arrays of densities and results ([n][3] each) lie r * U doubles
// apart; act[r] == 0 skips right-hand side r (act NULL: all run).  The default is one
// right-hand side.
struct Bat {
  int64_t A = 0;
  int64_t U = 0;
  const int* act = nullptr;
  int nb = 1;
};

// device tables for one precision and grid size
template <typename T>
struct DevTables {
  void* tw = nullptr;   // C2<T>[N]
  void* tw2 = nullptr;  // C2<T>[2N]
  void* mk = nullptr;   // C2<T>[N]
  T* sc = nullptr;      // [N]
  T* isc = nullptr;     // [N]
  T s0 = 0, s1 = 0, is0 = 0, is1 = 0;  // sc[0], sc[k > 0], isc[0], isc[k > 0]
  double* sig = nullptr;   // sigma_k = (2/h) sin(pi k / 2N), k < N
  double* sig2s = nullptr; // sigma_{k+1}^2, k < N
  T* sg2 = nullptr;        // sigma_k^2 in T
  T* sg2s = nullptr;       // sigma_{k+1}^2 in T
};

enum WeightKind { W_SCHUR = 0, W_RHS = 1 };

// ---- transforms
// pmask / xmask / mbit (optional, forward sparse inputs along axis 2 or 1): the input is zero
// outside the z-pencils (x, y) with bit mbit of pmask[x N + y] set (xmask[x]: or over y); tiles
// whose transform is then zero are written as zeros without being read
template <typename T>
hipError_t launch_pass(int N, int kind, int axis, const T* in, T* out, bool accumulate, const DevTables<T>& tb,
                       hipStream_t s, const Bat& bt = Bat(), const uint8_t* pmask = nullptr,
                       const uint8_t* xmask = nullptr, int mbit = -1);
// fused x-pass of the Schur operator for the three components (fwd x, weight, inverse x)
template <typename T>
hipError_t launch_xmid(int N, T* A0, T* A1, T* A2, double mu, const DevTables<T>& tb, hipStream_t s,
                       const Bat& bt = Bat());
// Forward z pass of the Schur matvec (A = DST-II_z v, B = DCT-II_z v) with the CG updates folded in:
//   ZF_PLAIN  v = r (x, d, q, scal, rpart unused)
//   ZF_FIRST  r -= scal[9] / N^3 (the mean of r given its sum), d = r, x = 0, v = d;
//             rpart[block] = partial r.r
//   ZF_FUSED  x += alpha d; r -= alpha (q - mean q); d = r + beta d (scal[1], scal[2], scal[3]);
//             v = d; rpart[block] = partial r.r of the updated r
// rpart holds zfwd_blocks(N, sizeof(T)) doubles.
//   ZF_FINAL  r += scal[1] d (written back), v = r
enum ZfwdMode { ZF_PLAIN = 0, ZF_FIRST = 1, ZF_FUSED = 2, ZF_FINAL = 3 };
template <typename T>
hipError_t launch_zfwd_cg(int N, int mode, T* x, T* r, T* d, const T* q, T* A, T* B, const double* scal,
                          double* rpart, const DevTables<T>& tb, hipStream_t s, const Bat& bt = Bat());
int zfwd_blocks(int N, int elem_size);
// q = DST-III_z(A) + DCT-III_z(B) + c d; per-block partial sums (d.q, q, d, q.q), 4 per block
template <typename T>
hipError_t launch_zinv_cg(int N, const T* A, const T* B, T* q, const T* d, double c, double* partials,
                          const DevTables<T>& tb, hipStream_t s, const Bat& bt = Bat());
// fused x pass of component m: right-hand side (fh = T_m,x in; out = C_m,x^T (-sigma/(mu Lambda)) fh)
// or back-substitution (out = T_m,x^T ((fh + sigma C_m,x in) / (mu Lambda)))
template <typename T>
hipError_t launch_xfuse(int N, int m, bool backsub, const T* in, T* fh, T* out, double mu, const DevTables<T>& tb,
                        hipStream_t s, const Bat& bt = Bat());
// y passes with two transforms per block: forward (out0 = DST-II_y(in0), out1 = DCT-II_y(in0)),
// inverse (out0 = DST-III_y(in0) + DCT-III_y(in1))
template <typename T>
hipError_t launch_ypair(int N, bool inverse, const T* in0, const T* in1, T* out0, T* out1, const DevTables<T>& tb,
                        hipStream_t s, const Bat& bt = Bat());
int zinv_blocks(int N, int elem_size);
// x += scal[idx] d
template <typename T>
hipError_t launch_axpy_scal(int64_t M, T* x, const T* d, const double* scal, int idx, hipStream_t s,
                            const Bat& bt = Bat());
// CG coefficients from the partial sums of the forward z pass (r.r, nr blocks) and of the
// inverse z pass (nz blocks of 4): scal[0] = |r_next|^2 (recurrence), [1] alpha, [2] beta,
// [3] mean q (Stokes), [7] r.r
hipError_t launch_cg_coef(const double* rpart, int nr, const double* zpart, int nz, double* scal, int stokes,
                          int64_t M, hipStream_t s, const Bat& bt = Bat(), double* hslot = nullptr);

// ---- reductions (float64, deterministic)
// scal layout: [0] |r_next|^2, [1] alpha, [2] beta, [3] mean q, [5] scratch sum, [6] aux, [7] r.r,
// [9] sum of the right-hand side
// R_SUM: the sum of the first of nper values per block; R_SUM1: of the second (nper <= 4)
enum ReduceOp { R_SUM = 2, R_RESNORM = 4, R_RESNORM0 = 5, R_SUM1 = 6 };
// (out, when given, is a work buffer like scal: it moves with the right-hand side in a batch)
// hdst (optional): the residual norm of R_RESNORM / R_RESNORM0 also goes to hdst[rhs]
// (a device address of pinned host memory)
hipError_t launch_reduce(const double* partials, int nparts, int nper, double* scal, int op, int stokes,
                         int64_t M, hipStream_t s, double* out = nullptr,
                         const Bat& bt = Bat(), double* hdst = nullptr);  // R_SUM: *out (or scal[5])
template <typename T>
hipError_t launch_dot_partials(int64_t M, const T* a, const T* b, double* partials, int nblocks, hipStream_t s);
template <typename T>
hipError_t launch_sum_partials(int64_t M, const T* a, double* partials, int nblocks, hipStream_t s,
                               const Bat& bt = Bat());
template <typename T>
hipError_t launch_add_scalar(int64_t M, T* a, const double* scal, int idx, double factor, hipStream_t s,
                             const Bat& bt = Bat());

// ---- elementwise
template <typename T>
hipError_t launch_fill(int64_t n, T* a, T v, hipStream_t s, const Bat& bt = Bat());
template <typename T>
hipError_t launch_axpby(int64_t n, T* y, double a, const T* x, double b, hipStream_t s);  // y = a x + b y

// ---- full-system residual of the MAC scheme (float64)
// r_u = F_u - (-mu lap u + G p), r_p = F_p - (D u + c p), internal layout
// mixed refinement: r32 = (float) F and partial sums of F (3 per block, nparts blocks)
hipError_t launch_refine_prep(int64_t M, const double* F, float* r32, double* partials, int nparts, hipStream_t s,
                              const Bat& bt = Bat());
// un, pn = u, p (+ 0 if first) + x32; r32 = float32 of the float64 residual F - A(un, pn) (pressure
// part minus *shift); partial sums.  norms_only (first round only): the partial sums alone,
// un, pn and r32 are not written (may be null).  fmask (optional, N^2 bytes): per z-pencil (x, y)
// bit c set where component c of F may be nonzero; F is read only there (zero elsewhere)
hipError_t launch_refine_residual(bool first, int N, double h, double mu, double c, const double* u, const double* p,
                                  const float* x32, const double* F, const double* shift, double* un, double* pn,
                                  float* r32, double* partials, int nparts, hipStream_t s, const Bat& bt = Bat(),
                                  bool norms_only = false, const uint8_t* fmask = nullptr);

// ---- surface stages (float64)
// jumps of every crossing (jmap component-major: jmap[(r * 18 + c) * T + t]) and the fit
// values of the control points (fitvals[18 cp + c]).  In a batch one thread group serves up to
// FJ_RHS right-hand sides, so the fit weights and jump maps are read once for all of them.
constexpr int FJ_RHS = 4;
hipError_t launch_fit_jump(int64_t T, const int64_t* nb_ptr, const int32_t* nb_idx, const double* fitw,
                           const double* jmap, const double* jfmap, const double* Fj, const double* phi,
                           const int64_t* cp_of, double* jumps, double* fitvals, hipStream_t s,
                           const Bat& bt = Bat());
hipError_t launch_interp_jump(int64_t n, const int64_t* cp_target, const double* fitvals, const double* emap,
                              const double* efmap, const double* Fj, double* ejump, hipStream_t s,
                              const Bat& bt = Bat());
// F[irr_node[r]] = correction of node r (assigned: each node appears once; F elsewhere untouched);
// with r32 != nullptr also r32[irr_node[r]] = (float) the same value and, over nparts blocks,
// partial sums (F_u.F_u, sum F_p, F_p.F_p) of the corrections (M = N^3 splits F_u from F_p)
hipError_t launch_correct(int64_t nirr, const int64_t* irr_node, const int64_t* irr_ptr, const int32_t* arm_t,
                          const int8_t* arm_o, const double* arm_a, const double* jumps, double* F, hipStream_t s,
                          float* r32 = nullptr, int64_t M = 0, double* partials = nullptr, int nparts = 0,
                          const Bat& bt = Bat());
// probes: out[r] = sum_{q<8} w[8r+q] u[idx[8r+q]], r < 3 m (trilinear)
hipError_t launch_interp8(int64_t m, const int64_t* idx, const double* w, const double* u, double* out, hipStream_t s);
hipError_t launch_stab(int64_t n, const int64_t* ptr, const int32_t* idx, const double* sw, const double* a,
                       const double* phi, double* out, hipStream_t s, const Bat& bt = Bat());
hipError_t launch_stab_T(int64_t n, const int64_t* ptr, const int32_t* row, const double* sw, const double* a,
                         const double* w, double* out, hipStream_t s);
hipError_t launch_interp(int64_t n, const int64_t* idx, const double* w, const double* u, const double* ejump,
                         double* out, hipStream_t s, const Bat& bt = Bat());
// the same with the velocity given by the float32 first-round solution x32 of the mixed solve
// (face 0 of each component at zero); N a power of two
hipError_t launch_interp_x32(int64_t n, const int64_t* idx, const double* w, const float* x32, int N,
                             const double* ejump, double* out, hipStream_t s, const Bat& bt = Bat());
// adjoint
hipError_t launch_interp_T(int64_t nnode, const int64_t* ptr, const int64_t* node, const int32_t* row,
                           const double* w, const double* wbar, double* ubar, hipStream_t s);
hipError_t launch_correct_T(int64_t T, const int64_t* ptr, const int64_t* node, const int8_t* slot, const double* a,
                            const double* Fbar, double* jbar, hipStream_t s);
hipError_t launch_jump_T(int64_t T, const int64_t* cp_of, const double* jmap, const double* emap,
                         const double* jbar, const double* wbar, double* fitbar, hipStream_t s);
hipError_t launch_fit_T(int64_t n, const int64_t* ptr, const int64_t* entry, const int32_t* target,
                        const double* fitw, const double* fitbar, double* phibar, hipStream_t s);
// layout conversion between the exported (N+1)-face layout and the internal one
hipError_t launch_export_u(int N, const double* u_int, double* u_ext, hipStream_t s);
hipError_t launch_import_u(int N, const double* u_ext, double* u_int, hipStream_t s);
hipError_t launch_scatter_add(int64_t n, const int64_t* idx, const double* v, double* F, hipStream_t s);
// *flag = tag if any a[i] is not finite (flag: a device address, pinned host memory in practice)
hipError_t launch_check_finite(int64_t n, const double* a, int* flag, int tag, hipStream_t s);
// out[i] = (To) in[i]
template <typename Ti, typename To>
hipError_t launch_convert(int64_t n, const Ti* in, To* out, hipStream_t s);

// ---- the DCT-II along x as a split-bfloat16 matrix product on the matrix cores (a measured
// alternative to the radix pass; float32 fields, N = 128, 256, 512)
bool gemm_pass_supported(int N);
// the hi and lo bfloat16 A-operand fragments of the orthonormal DCT-II matrix (2 N^2 values)
std::vector<uint16_t> gemm_dct2_fragments(int N);
hipError_t launch_gemm_dct2_x(int N, const float* in, float* out, const void* Cf, hipStream_t s);

}  // namespace kfbi
