// Host-side setup of the KFBI operator (Algorithm 1 step 1 of the paper, plus the sparse
// maps that the device kernels apply).  Plain C++17, float64 throughout.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/kfbi.h"

namespace kfbi {

// Grid ids: 0,1,2 = face grids T^1..T^3 (velocity component m), 3 = cell centres T^0 (p).
constexpr int GP = 3;

// Line families: for axis k the k-lines of T^0 (g = GP; they are also the k-lines of T^k)
// and of the two other face grids g = m != k.  Index f = 3 k + slot.
struct Family {
  int k;  // line axis
  int g;  // grid defining the transverse positions (GP or m != k)
};
Family family(int f);
int family_index(int k, int g);

// Second-order forward-mode number: value, gradient and Hessian (upper triangle
// 00,01,02,11,12,22) with respect to the three space coordinates.
struct HD {
  double v = 0, g[3] = {0, 0, 0}, h[6] = {0, 0, 0, 0, 0, 0};
};

struct LevelSet {
  kfbi_shape s;
  double bb_lo[3], bb_hi[3];
  explicit LevelSet(const kfbi_shape& shape);
  double value(double x, double y, double z) const;
  HD eval(double x, double y, double z) const;  // psi with exact gradient and Hessian
  bool inside(double x, double y, double z) const { return value(x, y, z) <= 0.0; }
};

struct Setup {
  // problem
  int N = 0;
  double lo = 0, hi = 0, h = 0;
  int pde = 0;
  double mu = 1, lam = 0;
  int64_t M = 0;  // N^3

  // node sides (1 = inside Omega), internal layout [x][y][z] of size N^3 per grid; for face
  // grid m the index along m is the face index a = 0..N-1 (face N lies on the box, outside)
  std::vector<uint8_t> side[4];

  // crossings ("targets"): all crossings of the nine families, family order, then lines
  // lexicographically, then ascending position
  int64_t T = 0;
  std::vector<int32_t> fam, l1, l2, jint;
  std::vector<double> pos, xyz, nrm, t1, t2, kap;  // xyz/nrm/t1/t2: 3 per target, kap: 4
  std::vector<int64_t> cp_of;                      // control-point index or -1
  std::vector<int64_t> cp_target;                  // crossing index of each control point
  int64_t n = 0;                                   // control points

  // least-squares fit: CSR over targets; 6 weights per neighbour entry
  std::vector<int64_t> nb_ptr;
  std::vector<int32_t> nb_idx;
  std::vector<double> fitw;

  // jump maps: 5 outputs per target x 18 fit inputs (slot layout: [[v]], d_k[[v]],
  // d_kk[[v]] of the component v the family serves, then [[p]], d_k[[p]] on T^0 families),
  // response to [[f]] (5 x 3), and the interpolation jump term per control point (3 x 18)
  std::vector<double> jmap, jfmap, emap;

  // corrections: CSR over irregular equation nodes; node = global index g*M + linear index
  std::vector<int64_t> irr_node, irr_ptr;
  std::vector<int32_t> arm_t;
  std::vector<int8_t> arm_o;   // 0 = velocity slots 0..2, 3 = pressure slots 3..4
  std::vector<double> arm_a;   // 3 coefficients per arm

  // interpolation: per (control point, component) 10 node indices (global, internal
  // layout) and weights; node side flags are folded into emap
  std::vector<int64_t> itp_idx;
  std::vector<double> itp_w;

  // transposes for the adjoint (deterministic gathers)
  std::vector<int64_t> uT_ptr, uT_node;  // interpolation^T: CSR over distinct grid nodes
  std::vector<int32_t> uT_row;           // row = 3*cp + m
  std::vector<double> uT_w;
  std::vector<int64_t> cT_ptr;           // corrections^T: CSR over targets
  std::vector<int64_t> cT_node;
  std::vector<int8_t> cT_slot;
  std::vector<double> cT_a;
  std::vector<int64_t> fT_ptr;           // fit^T: CSR over control points
  std::vector<int64_t> fT_entry;         // neighbour-entry index e (target found by search)
  std::vector<int32_t> fT_target;

  // average trace form: K phi += (1/2 - alpha)(phi - S phi) per control point and component,
  // alpha = exterior weight fraction of the interpolation stencil, S phi = least-squares
  // fitted value at the control point (before the density replaces it); CSR over control
  // points with its transpose
  std::vector<double> stab_a;            // 1/2 - alpha, 3 per control point
  std::vector<int64_t> sv_ptr;
  std::vector<int32_t> sv_idx;
  std::vector<double> sv_w;
  std::vector<int64_t> svT_ptr;
  std::vector<int32_t> svT_row;
  std::vector<double> svT_w;
};

// Builds everything; returns "" on success or an error message (prefixed "GEOM:" for
// geometry failures).
std::string build_setup(const kfbi_config& cfg, Setup& S);

// Jump relations at one surface point (exposed for the host unit test).  Inputs: frame
// n,t1,t2, curvature kap[2][2], fit values fv[6][3] (value, d1, d2, d11, d12, d22 per
// component), [[f]] F[3].  Output 34 values: [[u_i]] (3), d_k[[u_i]] (3i+k), d_k d_l [[u_i]]
// (12 + 9 i + 3 k + l, full 3x3), [[p]] (39), d_k [[p]] (40 + k).
void jump_point(int pde, double mu, double lam, const double n[3], const double t1[3],
                const double t2[3], const double kap[4], const double fv[18], const double F[3],
                double out[43]);

}  // namespace kfbi
