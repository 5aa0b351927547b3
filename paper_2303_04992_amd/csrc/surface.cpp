// Surface calculus of the KFBI setup: least-squares surface derivatives of the density and
// the interface jump relations, assembled into per-crossing linear maps.
//
// Paper: the correction terms (Sec. 4.3) and the interpolation jump function (Sec. 4.4) need
// the jumps of u, grad u, hess u, p and grad p at surface points, which the paper says follow
// from the interface conditions and the PDE without giving the derivation.
//
// Reading of the surface derivatives (the cited "equilibration" is not available): at a
// target x0 with frame (t1, t2, n), an unweighted least-squares quadratic in
// xi = (t1.(x-x0), t2.(x-x0))/h with basis [1, xi1, xi2, xi1^2/2, xi1 xi2, xi2^2/2] over the
// control points within 2.5h (grown by 0.5h up to 4h until there are 12) whose normals
// satisfy n.n0 >= 0.5; at a control point the value is the density itself.
//
// Jump relations (derivation in closed form; w = d[[u]]/dn):
//  first order   [[grad u]] = w n^T + sum_a Phi_a t_a^T, t_a.w = -n.Phi_a (zero traction
//                jump), Stokes n.w = -sum_a t_a.Phi_a, [[p]] = 2 mu n.w; Navier
//                n.w = -lambda s/(lambda+2mu), [[p]] = -(lambda+mu)[[div u]];
//  second order  tangential block from the Monge patch, V_ab = Phi_ab - kappa_ab w; mixed
//                block from the tangential derivative of the traction condition (and of
//                [[div u]] = 0 for Stokes); normal block from the momentum jump (and the
//                normal derivative of [[div u]] = 0 for Stokes).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "setup.h"

namespace kfbi {

static inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

void jump_point(int pde, double mu, double lam, const double n[3], const double t1[3], const double t2[3],
                const double kap[4], const double fv[18], const double F[3], double out[43]) {
  const double* t[2] = {t1, t2};
  // fit values: Phi[i] = fv[0*3+i], Phi_a[a][i] = fv[(1+a)*3+i], Phi_ab by (11,12,22)
  double Phi[3], Pa[2][3], Pab[3][3];
  for (int i = 0; i < 3; ++i) {
    Phi[i] = fv[i];
    Pa[0][i] = fv[3 + i];
    Pa[1][i] = fv[6 + i];
    Pab[0][i] = fv[9 + i];
    Pab[1][i] = fv[12 + i];
    Pab[2][i] = fv[15 + i];
  }
  // ---- first order (traction jump zero)
  double s = dot3(t[0], Pa[0]) + dot3(t[1], Pa[1]);
  double wt[2] = {-dot3(n, Pa[0]), -dot3(n, Pa[1])};
  double wn, jp, jdiv = 0;
  if (pde == KFBI_STOKES) {
    wn = -s;
    jp = 2.0 * mu * wn;
  } else {
    wn = -lam * s / (lam + 2.0 * mu);
    jdiv = wn + s;
    jp = -(lam + mu) * jdiv;
  }
  double w[3], Gu[3][3], sig[3][3];
  for (int i = 0; i < 3; ++i) w[i] = wn * n[i] + wt[0] * t[0][i] + wt[1] * t[1][i];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) Gu[i][k] = w[i] * n[k] + Pa[0][i] * t[0][k] + Pa[1][i] * t[1][k];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) {
      double diag = (i == k) ? (pde == KFBI_STOKES ? -jp : lam * jdiv) : 0.0;
      sig[i][k] = diag + mu * (Gu[i][k] + Gu[k][i]);
    }
  // ---- second order: tangential-tangential block V[a][b][i]
  double V[2][2][3];
  const int abi[2][2] = {{0, 1}, {1, 2}};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int i = 0; i < 3; ++i) V[a][b][i] = Pab[abi[a][b]][i] - kap[2 * a + b] * w[i];
  // ---- mixed block
  double Van[2][3], pia[2] = {0, 0}, dla[2] = {0, 0};
  for (int a = 0; a < 2; ++a) {
    double Rp[3] = {0, 0, 0};  // sum_b kappa_ab [[sigma]] t_b (traction derivative zero)
    for (int b = 0; b < 2; ++b)
      for (int i = 0; i < 3; ++i) Rp[i] += kap[2 * a + b] * dot3(sig[i], t[b]);
    double tV = dot3(t[0], V[a][0]) + dot3(t[1], V[a][1]);
    double nVan;
    if (pde == KFBI_STOKES) {
      nVan = -tV;
      pia[a] = 2.0 * mu * nVan - dot3(n, Rp);
    } else {
      nVan = (dot3(n, Rp) - lam * tV) / (lam + 2.0 * mu);
      dla[a] = tV + nVan;
    }
    double tc[2];
    for (int c = 0; c < 2; ++c) tc[c] = dot3(t[c], Rp) / mu - dot3(n, V[a][c]);
    for (int i = 0; i < 3; ++i) Van[a][i] = nVan * n[i] + tc[0] * t[0][i] + tc[1] * t[1][i];
  }
  // ---- normal block
  double S12[3];
  for (int i = 0; i < 3; ++i) S12[i] = V[0][0][i] + V[1][1][i];
  double tVan = dot3(t[0], Van[0]) + dot3(t[1], Van[1]);
  double Vnn[3], gp[3];
  if (pde == KFBI_STOKES) {
    double nVnn = -tVan;
    double pin = mu * (nVnn + dot3(n, S12)) + dot3(n, F);
    for (int i = 0; i < 3; ++i) {
      gp[i] = pia[0] * t[0][i] + pia[1] * t[1][i] + pin * n[i];
      Vnn[i] = (gp[i] - F[i]) / mu - S12[i];
    }
  } else {
    double nVnn = -(dot3(n, F) + mu * dot3(n, S12) + (lam + mu) * tVan) / (lam + 2.0 * mu);
    double dn = tVan + nVnn;
    for (int i = 0; i < 3; ++i) {
      double g = dla[0] * t[0][i] + dla[1] * t[1][i] + dn * n[i];
      Vnn[i] = -(F[i] + (lam + mu) * g) / mu - S12[i];
      gp[i] = -(lam + mu) * g;
    }
  }
  // ---- assemble
  for (int i = 0; i < 3; ++i) out[i] = Phi[i];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) out[3 + 3 * i + k] = Gu[i][k];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) {
        double v = 0;
        for (int a = 0; a < 2; ++a) {
          for (int b = 0; b < 2; ++b) v += V[a][b][i] * t[a][k] * t[b][l];
          v += Van[a][i] * (t[a][k] * n[l] + n[k] * t[a][l]);
        }
        v += Vnn[i] * n[k] * n[l];
        out[12 + 9 * i + 3 * k + l] = v;
      }
  out[39] = jp;
  for (int k = 0; k < 3; ++k) out[40 + k] = gp[k];
}

// ---------------------------------------------------------------------------------------
// neighbour search (cell hash over the box) and least-squares weights
// ---------------------------------------------------------------------------------------
// Householder QR of A (K x 6, row-major); returns the pseudo-inverse P (6 x K).
static bool lsq_pinv(int K, std::vector<double>& A, double* P) {
  const int C = 6;
  std::vector<double> Q(K * K, 0.0);
  for (int i = 0; i < K; ++i) Q[i * K + i] = 1.0;
  std::vector<double> v(K);
  for (int j = 0; j < C; ++j) {
    double nrm = 0;
    for (int i = j; i < K; ++i) nrm += A[i * C + j] * A[i * C + j];
    nrm = std::sqrt(nrm);
    if (nrm == 0) return false;
    double alpha = (A[j * C + j] > 0) ? -nrm : nrm;
    for (int i = 0; i < K; ++i) v[i] = (i < j) ? 0.0 : A[i * C + j];
    v[j] -= alpha;
    double vn = 0;
    for (int i = j; i < K; ++i) vn += v[i] * v[i];
    if (vn == 0) continue;
    // A <- (I - 2 v v^T / vn) A
    for (int c = j; c < C; ++c) {
      double s = 0;
      for (int i = j; i < K; ++i) s += v[i] * A[i * C + c];
      s = 2.0 * s / vn;
      for (int i = j; i < K; ++i) A[i * C + c] -= s * v[i];
    }
    // Q^T accumulated as rows: Qt <- H Qt
    for (int c = 0; c < K; ++c) {
      double s = 0;
      for (int i = j; i < K; ++i) s += v[i] * Q[i * K + c];
      s = 2.0 * s / vn;
      for (int i = j; i < K; ++i) Q[i * K + c] -= s * v[i];
    }
  }
  // P = R^{-1} (Q^T)[0:6, :]
  for (int c = 0; c < K; ++c) {
    double y[6];
    for (int r = C - 1; r >= 0; --r) {
      double s = Q[r * K + c];
      for (int q = r + 1; q < C; ++q) s -= A[r * C + q] * y[q];
      if (A[r * C + r] == 0) return false;
      y[r] = s / A[r * C + r];
    }
    for (int r = 0; r < C; ++r) P[r * K + c] = y[r];
  }
  return true;
}

std::string build_fits(Setup& S) {
  const int64_t n = S.n, T = S.T;
  const double h = S.h;
  // cell hash over the bounding box of the control points
  double blo[3] = {1e300, 1e300, 1e300}, bhi[3] = {-1e300, -1e300, -1e300};
  for (int64_t c = 0; c < n; ++c)
    for (int d = 0; d < 3; ++d) {
      double x = S.xyz[3 * S.cp_target[c] + d];
      blo[d] = std::min(blo[d], x);
      bhi[d] = std::max(bhi[d], x);
    }
  int dims[3];
  for (int d = 0; d < 3; ++d) dims[d] = std::max(1, (int)std::floor((bhi[d] - blo[d]) / h) + 1);
  const int64_t ncell = (int64_t)dims[0] * dims[1] * dims[2];
  auto cell_of = [&](const double* x, int* ci) {
    for (int d = 0; d < 3; ++d) ci[d] = (int)std::floor((x[d] - blo[d]) / h);
  };
  std::vector<int64_t> head(ncell + 1, 0);
  std::vector<int64_t> cid(n);
  for (int64_t c = 0; c < n; ++c) {
    int ci[3];
    cell_of(&S.xyz[3 * S.cp_target[c]], ci);
    for (int d = 0; d < 3; ++d) ci[d] = std::min(std::max(ci[d], 0), dims[d] - 1);
    cid[c] = ((int64_t)ci[0] * dims[1] + ci[1]) * dims[2] + ci[2];
    head[cid[c] + 1]++;
  }
  for (int64_t i = 0; i < ncell; ++i) head[i + 1] += head[i];
  std::vector<int64_t> fill(head.begin(), head.end() - 1), items(n);
  for (int64_t c = 0; c < n; ++c) items[fill[cid[c]]++] = c;  // ascending within a cell

  std::vector<std::vector<int32_t>> nb(T);
  std::vector<std::vector<double>> W(T), raw0(T);  // raw0: fitted value weights (control targets)
  std::string err;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t t = 0; t < T; ++t) {
    const double* x0 = &S.xyz[3 * t];
    const double* n0 = &S.nrm[3 * t];
    std::vector<int32_t> L;
    double r = 2.5 * h + 1e-9 * h;
    while (true) {
      L.clear();
      int rc = (int)std::ceil(r / h) + 1;
      int ci[3];
      cell_of(x0, ci);
      for (int a = ci[0] - rc; a <= ci[0] + rc; ++a) {
        if (a < 0 || a >= dims[0]) continue;
        for (int b = ci[1] - rc; b <= ci[1] + rc; ++b) {
          if (b < 0 || b >= dims[1]) continue;
          for (int c = ci[2] - rc; c <= ci[2] + rc; ++c) {
            if (c < 0 || c >= dims[2]) continue;
            int64_t id = ((int64_t)a * dims[1] + b) * dims[2] + c;
            for (int64_t q = head[id]; q < head[id + 1]; ++q) {
              int64_t cp = items[q];
              const double* x = &S.xyz[3 * S.cp_target[cp]];
              double dx = x[0] - x0[0], dy = x[1] - x0[1], dz = x[2] - x0[2];
              if (std::sqrt(dx * dx + dy * dy + dz * dz) <= r &&
                  dot3(&S.nrm[3 * S.cp_target[cp]], n0) >= 0.5)
                L.push_back((int32_t)cp);
            }
          }
        }
      }
      if (L.size() >= 12) break;
      r += 0.5 * h;
      if (r > 4.0 * h + 2e-9 * h) {
#pragma omp critical
        err = "GEOM: fewer than 12 control points within 4h of a crossing";
        break;
      }
    }
    if (L.size() < 12) continue;
    std::sort(L.begin(), L.end());
    const int K = (int)L.size();
    std::vector<double> A(K * 6), P(6 * K);
    const double* a1 = &S.t1[3 * t];
    const double* a2 = &S.t2[3 * t];
    for (int q = 0; q < K; ++q) {
      const double* x = &S.xyz[3 * S.cp_target[L[q]]];
      double d[3] = {x[0] - x0[0], x[1] - x0[1], x[2] - x0[2]};
      double u = dot3(d, a1) / h, v = dot3(d, a2) / h;
      double row[6] = {1.0, u, v, 0.5 * u * u, u * v, 0.5 * v * v};
      for (int c = 0; c < 6; ++c) A[q * 6 + c] = row[c];
    }
    if (!lsq_pinv(K, A, P.data())) {
#pragma omp critical
      err = "GEOM: singular least-squares fit";
      continue;
    }
    const double sc[6] = {1.0, 1.0 / h, 1.0 / h, 1.0 / (h * h), 1.0 / (h * h), 1.0 / (h * h)};
    for (int r2 = 0; r2 < 6; ++r2)
      for (int q = 0; q < K; ++q) P[r2 * K + q] *= sc[r2];
    if (S.cp_of[t] >= 0) {
      raw0[t].assign(P.begin(), P.begin() + K);
      for (int q = 0; q < K; ++q) P[q] = (L[q] == S.cp_of[t]) ? 1.0 : 0.0;
    }
    nb[t] = L;
    W[t].assign(6 * K, 0.0);
    for (int q = 0; q < K; ++q)
      for (int r2 = 0; r2 < 6; ++r2) W[t][6 * q + r2] = P[r2 * K + q];
  }
  if (!err.empty()) return err;
  S.nb_ptr.assign(T + 1, 0);
  for (int64_t t = 0; t < T; ++t) S.nb_ptr[t + 1] = S.nb_ptr[t] + (int64_t)nb[t].size();
  S.nb_idx.resize(S.nb_ptr[T]);
  S.fitw.resize(6 * S.nb_ptr[T]);
  for (int64_t t = 0; t < T; ++t) {
    std::copy(nb[t].begin(), nb[t].end(), S.nb_idx.begin() + S.nb_ptr[t]);
    std::copy(W[t].begin(), W[t].end(), S.fitw.begin() + 6 * S.nb_ptr[t]);
  }
  // fitted-value rows of the control points and their transpose
  S.sv_ptr.assign(n + 1, 0);
  for (int64_t c = 0; c < n; ++c) S.sv_ptr[c + 1] = S.sv_ptr[c] + (int64_t)nb[S.cp_target[c]].size();
  S.sv_idx.resize(S.sv_ptr[n]);
  S.sv_w.resize(S.sv_ptr[n]);
  S.svT_ptr.assign(n + 1, 0);
  for (int64_t c = 0; c < n; ++c) {
    const int64_t t = S.cp_target[c];
    std::copy(nb[t].begin(), nb[t].end(), S.sv_idx.begin() + S.sv_ptr[c]);
    std::copy(raw0[t].begin(), raw0[t].end(), S.sv_w.begin() + S.sv_ptr[c]);
    for (int32_t j : nb[t]) S.svT_ptr[j + 1]++;
  }
  for (int64_t j = 0; j < n; ++j) S.svT_ptr[j + 1] += S.svT_ptr[j];
  S.svT_row.resize(S.sv_ptr[n]);
  S.svT_w.resize(S.sv_ptr[n]);
  std::vector<int64_t> pos(S.svT_ptr.begin(), S.svT_ptr.end() - 1);
  for (int64_t c = 0; c < n; ++c)  // ascending c within each transposed row
    for (int64_t e = S.sv_ptr[c]; e < S.sv_ptr[c + 1]; ++e) {
      const int64_t q = pos[S.sv_idx[e]]++;
      S.svT_row[q] = (int32_t)c;
      S.svT_w[q] = S.sv_w[e];
    }
  return "";
}

// per-target jump maps (5 slots x 18 fit inputs, 5 x 3 force inputs)
void build_jump_maps(Setup& S) {
  const int64_t T = S.T;
  S.jmap.assign(T * 5 * 18, 0.0);
  S.jfmap.assign(T * 5 * 3, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < T; ++t) {
    Family F = family(S.fam[t]);
    int v = (F.g == GP) ? F.k : F.g;  // velocity component served by this line family
    int k = F.k;
    int rows[5] = {v, 3 + 3 * v + k, 12 + 9 * v + 3 * k + k, 39, 40 + k};
    int nrow = (F.g == GP) ? 5 : 3;
    double fv[18], Fz[3] = {0, 0, 0}, out[43];
    for (int c = 0; c < 18; ++c) {
      std::memset(fv, 0, sizeof(fv));
      fv[c] = 1.0;
      jump_point(S.pde, S.mu, S.lam, &S.nrm[3 * t], &S.t1[3 * t], &S.t2[3 * t], &S.kap[4 * t], fv, Fz, out);
      for (int r = 0; r < nrow; ++r) S.jmap[(t * 5 + r) * 18 + c] = out[rows[r]];
    }
    std::memset(fv, 0, sizeof(fv));
    for (int c = 0; c < 3; ++c) {
      double Fu[3] = {0, 0, 0};
      Fu[c] = 1.0;
      jump_point(S.pde, S.mu, S.lam, &S.nrm[3 * t], &S.t1[3 * t], &S.t2[3 * t], &S.kap[4 * t], fv, Fu, out);
      for (int r = 0; r < nrow; ++r) S.jfmap[(t * 5 + r) * 3 + c] = out[rows[r]];
    }
  }
}

}  // namespace kfbi
