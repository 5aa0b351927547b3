// Assembly of the correction arms (Sec. 4.3), the ten-node interpolation (Sec. 4.4) and the
// transposed maps used by the adjoint.
//
// Correction rule (reading; it reproduces cases 1-3 and the pressure term of case 4 as
// printed, and fixes the sign of the velocity term of case 4 so that constant densities are
// reproduced exactly): an equation at z0 whose stencil coefficient c_q multiplies a node z_q
// on the other side of the surface gets C = -s(z0) c_q D_q on its right-hand side, with
// s = +1 in Omega and -1 outside, D_q = [[v]] + xi [[v_k]] + xi^2/2 [[v_kk]] for a velocity
// node, [[p]] + xi [[p_k]] for a pressure node, at the crossing r on the arm, xi = (z_q - r)_k.
//
// Interpolation stencil (reading of the ten closest nodes): z0 = nearest node of T^m,
// s = sign(x - z0) (0 -> +1), nodes z0, z0 +- h e_k, z0 + h(s1 e1 + s2 e2),
// z0 + h(s1 e1 + s3 e3), z0 + h(s2 e2 + s3 e3); quadratic basis in d = (z - x)/h:
// [1, d1, d2, d3, d1^2/2, d2^2/2, d3^2/2, d2 d3, d1 d3, d1 d2]; weights = first row of the
// inverse of the 10 x 10 basis matrix.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "setup.h"

namespace kfbi {

std::string build_fits(Setup& S);
void build_jump_maps(Setup& S);
void build_geometry(const kfbi_config& cfg, Setup& S);

static inline int64_t lin(const Setup& S, int i, int j, int k) { return ((int64_t)i * S.N + j) * S.N + k; }

static std::string build_corrections(Setup& S) {
  const int N = S.N;
  const double h = S.h, lo = S.lo, mu = S.mu;
  std::unordered_map<uint64_t, int32_t> look;
  look.reserve(S.T * 2);
  auto key = [&](int f, int a, int b, int j) -> uint64_t {
    return (((uint64_t)f * (N + 1) + a) * (N + 1) + b) * (uint64_t)(2 * N + 1) + j;
  };
  for (int64_t t = 0; t < S.T; ++t) look[key(S.fam[t], S.l1[t], S.l2[t], S.jint[t])] = (int32_t)t;

  struct Arm {
    int32_t t;
    int8_t o;
    double a[3];
  };
  std::vector<std::pair<int64_t, std::vector<Arm>>> eqs;
  std::string err;
  // node index range to scan: bounding box of the crossings +- 2 cells
  int blo[3], bhi[3];
  for (int d = 0; d < 3; ++d) {
    double mn = 1e300, mx = -1e300;
    for (int64_t t = 0; t < S.T; ++t) {
      mn = std::min(mn, S.xyz[3 * t + d]);
      mx = std::max(mx, S.xyz[3 * t + d]);
    }
    blo[d] = std::max(0, (int)std::floor((mn - lo) / h) - 2);
    bhi[d] = std::min(N - 1, (int)std::ceil((mx - lo) / h) + 2);
  }
  for (int g = 0; g < 4; ++g) {
    const uint8_t* sd = S.side[g].data();
    for (int i = blo[0]; i <= bhi[0]; ++i)
      for (int j = blo[1]; j <= bhi[1]; ++j)
        for (int k = blo[2]; k <= bhi[2]; ++k) {
          int idx[3] = {i, j, k};
          if (g < 3 && idx[g] == 0) continue;  // box face: no equation
          const bool in0 = sd[lin(S, i, j, k)] != 0;
          const double s0 = in0 ? 1.0 : -1.0;
          double z0[3];
          for (int d = 0; d < 3; ++d) z0[d] = (d == g) ? lo + idx[d] * h : lo + (idx[d] + 0.5) * h;
          std::vector<Arm> arms;
          auto add_arm = [&](int d, int sgn, double step, int fam_g, int nb_grid, const int* nbidx, double coef,
                             int8_t o) {
            for (int q = 0; q < 3; ++q)
              if (nbidx[q] < 0 || nbidx[q] >= N) return;  // ghost / box face: never crossed
            bool in1 = S.side[nb_grid][lin(S, nbidx[0], nbidx[1], nbidx[2])] != 0;
            if (in1 == in0) return;
            double zq = z0[d] + sgn * step * h;
            int ja = (int)std::lround((std::min(z0[d], zq) - lo) / (0.5 * h));
            int jb = (int)std::lround((std::max(z0[d], zq) - lo) / (0.5 * h));
            int f = family_index(d, fam_g);
            int ax[2], c = 0;
            for (int e = 0; e < 3; ++e)
              if (e != d) ax[c++] = e;
            int32_t t = -1;
            for (int jj = ja; jj < jb && t < 0; ++jj) {
              auto it = look.find(key(f, idx[ax[0]], idx[ax[1]], jj));
              if (it != look.end()) t = it->second;
            }
            if (t < 0) {
              err = "GEOM: crossed stencil arm without a crossing";
              return;
            }
            double xi = zq - S.pos[t];
            double cc = -s0 * coef;
            Arm A{t, o, {cc, cc * xi, (o == 0) ? 0.5 * cc * xi * xi : 0.0}};
            arms.push_back(A);
          };
          if (g < 3) {
            const int m = g;
            for (int d = 0; d < 3; ++d)
              for (int sgn = -1; sgn <= 1; sgn += 2) {
                int nb[3] = {i, j, k};
                nb[d] += sgn;
                add_arm(d, sgn, 1.0, d == m ? GP : m, m, nb, -mu / (h * h), 0);
              }
            // pressure gradient: p[a-1] at -h/2 (coeff -1/h), p[a] at +h/2 (coeff +1/h)
            for (int sgn = -1; sgn <= 1; sgn += 2) {
              int nb[3] = {i, j, k};
              if (sgn < 0) nb[m] -= 1;
              add_arm(m, sgn, 0.5, GP, GP, nb, sgn / h, 3);
            }
          } else {
            // continuity: face a (coeff -1/h) at -h/2 and face a+1 (coeff +1/h) at +h/2
            for (int d = 0; d < 3; ++d)
              for (int sgn = -1; sgn <= 1; sgn += 2) {
                int nb[3] = {i, j, k};
                if (sgn > 0) nb[d] += 1;
                add_arm(d, sgn, 0.5, GP, d, nb, sgn / h, 0);
              }
          }
          if (!err.empty()) return err;
          if (!arms.empty()) eqs.push_back({(int64_t)g * S.M + lin(S, i, j, k), std::move(arms)});
        }
  }
  std::sort(eqs.begin(), eqs.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  S.irr_node.clear();
  S.irr_ptr.assign(1, 0);
  S.arm_t.clear();
  S.arm_o.clear();
  S.arm_a.clear();
  for (auto& e : eqs) {
    S.irr_node.push_back(e.first);
    for (auto& A : e.second) {
      S.arm_t.push_back(A.t);
      S.arm_o.push_back(A.o);
      for (int q = 0; q < 3; ++q) S.arm_a.push_back(A.a[q]);
    }
    S.irr_ptr.push_back((int64_t)S.arm_t.size());
  }
  // transpose: per target, entries (node, slot, coefficient)
  std::vector<std::vector<std::tuple<int64_t, int8_t, double>>> per(S.T);
  for (size_t r = 0; r < S.irr_node.size(); ++r)
    for (int64_t q = S.irr_ptr[r]; q < S.irr_ptr[r + 1]; ++q) {
      int32_t t = S.arm_t[q];
      int8_t o = S.arm_o[q];
      int ns = (o == 0) ? 3 : 2;
      for (int s = 0; s < ns; ++s) per[t].emplace_back(S.irr_node[r], (int8_t)(o + s), S.arm_a[3 * q + s]);
    }
  S.cT_ptr.assign(S.T + 1, 0);
  for (int64_t t = 0; t < S.T; ++t) S.cT_ptr[t + 1] = S.cT_ptr[t] + (int64_t)per[t].size();
  S.cT_node.resize(S.cT_ptr[S.T]);
  S.cT_slot.resize(S.cT_ptr[S.T]);
  S.cT_a.resize(S.cT_ptr[S.T]);
  for (int64_t t = 0; t < S.T; ++t) {
    int64_t o = S.cT_ptr[t];
    for (auto& e : per[t]) {
      S.cT_node[o] = std::get<0>(e);
      S.cT_slot[o] = std::get<1>(e);
      S.cT_a[o] = std::get<2>(e);
      ++o;
    }
  }
  return "";
}

// solve V^T w = e0 for the 10 x 10 basis matrix V (LU with partial pivoting)
static bool first_row_of_inverse(double V[10][10], double w[10]) {
  double A[10][11];
  for (int r = 0; r < 10; ++r) {
    for (int c = 0; c < 10; ++c) A[r][c] = V[c][r];
    A[r][10] = (r == 0) ? 1.0 : 0.0;
  }
  for (int c = 0; c < 10; ++c) {
    int p = c;
    for (int r = c + 1; r < 10; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[p][c])) p = r;
    if (A[p][c] == 0) return false;
    if (p != c)
      for (int q = 0; q < 11; ++q) std::swap(A[p][q], A[c][q]);
    for (int r = c + 1; r < 10; ++r) {
      double f = A[r][c] / A[c][c];
      for (int q = c; q < 11; ++q) A[r][q] -= f * A[c][q];
    }
  }
  for (int r = 9; r >= 0; --r) {
    double s = A[r][10];
    for (int q = r + 1; q < 10; ++q) s -= A[r][q] * w[q];
    w[r] = s / A[r][r];
  }
  return true;
}

static std::string build_interpolation(Setup& S) {
  const int N = S.N;
  const double h = S.h, lo = S.lo;
  const int64_t n = S.n;
  S.itp_idx.assign(n * 30, 0);
  S.itp_w.assign(n * 30, 0.0);
  S.emap.assign(n * 3 * 18, 0.0);
  S.stab_a.assign(n * 3, 0.5);
  std::vector<double> efmap(n * 9, 0.0);
  std::string err;
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < n; ++c) {
    const int64_t t = S.cp_target[c];
    const double* x = &S.xyz[3 * t];
    // jump responses at the control point to the 18 fit inputs and 3 force inputs
    double resp[21][43];
    for (int q = 0; q < 21; ++q) {
      double fv[18] = {0}, F[3] = {0, 0, 0};
      if (q < 18)
        fv[q] = 1.0;
      else
        F[q - 18] = 1.0;
      jump_point(S.pde, S.mu, S.lam, &S.nrm[3 * t], &S.t1[3 * t], &S.t2[3 * t], &S.kap[4 * t], fv, F, resp[q]);
    }
    for (int m = 0; m < 3; ++m) {
      double off[3];
      int z0[3], s[3];
      for (int d = 0; d < 3; ++d) {
        off[d] = (d == m) ? 0.0 : 0.5;
        z0[d] = (int)std::floor((x[d] - lo) / h - off[d] + 0.5);
        double zc = lo + (z0[d] + off[d]) * h;
        s[d] = (x[d] - zc >= 0) ? 1 : -1;
      }
      int nodes[10][3];
      for (int q = 0; q < 10; ++q)
        for (int d = 0; d < 3; ++d) nodes[q][d] = z0[d];
      for (int k = 0; k < 3; ++k) {
        nodes[1 + 2 * k][k] -= 1;
        nodes[2 + 2 * k][k] += 1;
      }
      nodes[7][0] += s[0];
      nodes[7][1] += s[1];
      nodes[8][0] += s[0];
      nodes[8][2] += s[2];
      nodes[9][1] += s[1];
      nodes[9][2] += s[2];
      double V[10][10], dz[10][3];
      bool ok = true;
      for (int q = 0; q < 10; ++q) {
        for (int d = 0; d < 3; ++d) {
          if (nodes[q][d] < 0 || nodes[q][d] >= N) ok = false;
          dz[q][d] = lo + (nodes[q][d] + off[d]) * h - x[d];
        }
        if (nodes[q][m] < 1) ok = false;
        double d1 = dz[q][0] / h, d2 = dz[q][1] / h, d3 = dz[q][2] / h;
        double row[10] = {1, d1, d2, d3, 0.5 * d1 * d1, 0.5 * d2 * d2, 0.5 * d3 * d3, d2 * d3, d1 * d3, d1 * d2};
        for (int r = 0; r < 10; ++r) V[q][r] = row[r];
      }
      double w[10];
      if (!ok || !first_row_of_inverse(V, w)) {
#pragma omp critical
        err = "GEOM: interpolation stencil leaves the interior nodes";
        continue;
      }
      for (int q = 0; q < 10; ++q) {
        int64_t li = lin(S, nodes[q][0], nodes[q][1], nodes[q][2]);
        S.itp_idx[(c * 3 + m) * 10 + q] = (int64_t)m * S.M + li;
        S.itp_w[(c * 3 + m) * 10 + q] = w[q];
        if (S.side[m][li]) continue;  // interior node: no jump term
        S.stab_a[c * 3 + m] -= w[q];  // exterior weight fraction
        for (int in = 0; in < 21; ++in) {
          const double* o = resp[in];
          double J = o[m];
          for (int k = 0; k < 3; ++k) {
            J += dz[q][k] * o[3 + 3 * m + k];
            for (int l = 0; l < 3; ++l) J += 0.5 * dz[q][k] * dz[q][l] * o[12 + 9 * m + 3 * k + l];
          }
          if (in < 18)
            S.emap[(c * 3 + m) * 18 + in] += w[q] * J;
          else
            efmap[(c * 3 + m) * 3 + (in - 18)] += w[q] * J;
        }
      }
    }
  }
  if (!err.empty()) return err;
  S.emap.insert(S.emap.end(), efmap.begin(), efmap.end());  // n*54 fit part, then n*9 force part
  // transpose: CSR over distinct grid nodes
  std::vector<std::tuple<int64_t, int32_t, double>> ent;
  ent.reserve(n * 30);
  for (int64_t r = 0; r < n * 3; ++r)
    for (int q = 0; q < 10; ++q) ent.emplace_back(S.itp_idx[r * 10 + q], (int32_t)r, S.itp_w[r * 10 + q]);
  std::sort(ent.begin(), ent.end());
  S.uT_ptr.assign(1, 0);
  S.uT_node.clear();
  S.uT_row.clear();
  S.uT_w.clear();
  for (size_t e = 0; e < ent.size(); ++e) {
    if (e == 0 || std::get<0>(ent[e]) != std::get<0>(ent[e - 1])) {
      if (e > 0) S.uT_ptr.push_back((int64_t)e);
      S.uT_node.push_back(std::get<0>(ent[e]));
    }
    S.uT_row.push_back(std::get<1>(ent[e]));
    S.uT_w.push_back(std::get<2>(ent[e]));
  }
  S.uT_ptr.push_back((int64_t)ent.size());
  return "";
}

static void build_fit_transpose(Setup& S) {
  std::vector<std::vector<std::pair<int64_t, int32_t>>> per(S.n);
  for (int64_t t = 0; t < S.T; ++t)
    for (int64_t e = S.nb_ptr[t]; e < S.nb_ptr[t + 1]; ++e) per[S.nb_idx[e]].emplace_back(e, (int32_t)t);
  S.fT_ptr.assign(S.n + 1, 0);
  for (int64_t c = 0; c < S.n; ++c) S.fT_ptr[c + 1] = S.fT_ptr[c] + (int64_t)per[c].size();
  S.fT_entry.resize(S.fT_ptr[S.n]);
  S.fT_target.resize(S.fT_ptr[S.n]);
  for (int64_t c = 0; c < S.n; ++c) {
    int64_t o = S.fT_ptr[c];
    for (auto& p : per[c]) {
      S.fT_entry[o] = p.first;
      S.fT_target[o] = p.second;
      ++o;
    }
  }
}

std::string build_setup(const kfbi_config& cfg, Setup& S) {
  S.N = cfg.N;
  S.lo = cfg.lo;
  S.hi = cfg.hi;
  S.h = (cfg.hi - cfg.lo) / cfg.N;
  S.pde = cfg.pde;
  S.mu = cfg.mu;
  S.lam = cfg.lambda;
  S.M = (int64_t)cfg.N * cfg.N * cfg.N;
  build_geometry(cfg, S);
  if (S.n == 0) return "GEOM: no control points (surface outside the box or not resolved)";
  std::string e = build_fits(S);
  if (!e.empty()) return e;
  build_jump_maps(S);
  e = build_corrections(S);
  if (!e.empty()) return e;
  e = build_interpolation(S);
  if (!e.empty()) return e;
  build_fit_transpose(S);
  return "";
}

}  // namespace kfbi
