// Geometry of the KFBI setup: level sets with exact derivatives (second-order forward mode),
// node classification, crossings of the surface with the nine grid-line families, control
// points and local frames.
//
// Paper: Sec. 4.2 (box, grids T^0..T^3), Algorithm 1 step 1 (inside/outside marks,
// intersections with grid lines, normal and tangential directions), Sec. 3 (control points
// are intersections of the surface with grid lines; primary points).
//
// Readings (the paper leaves these open): Omega = {psi <= 0}, n = grad psi / |grad psi|.
// Crossings on a line are found from sign changes of (psi <= 0) between consecutive points
// of the half-step lattice lo + j h/2 and located by bisection until the bracket cannot
// shrink (midpoint of the final bracket).  Control points: crossings on the T^0 families
// with |n_k| >= (1 - 1e-12) max |n|.  Frame: t1 = normalise(e_j x n), j = argmin |n_j|
// (first on ties), t2 = n x t1; curvature kappa_ab = -t_a.(hess psi) t_b / |grad psi|.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "setup.h"

namespace kfbi {

Family family(int f) {
  int k = f / 3, s = f % 3;
  if (s == 0) return {k, GP};
  int others[2], c = 0;
  for (int m = 0; m < 3; ++m)
    if (m != k) others[c++] = m;
  return {k, others[s - 1]};
}

int family_index(int k, int g) {
  for (int s = 0; s < 3; ++s) {
    Family F = family(3 * k + s);
    if (F.g == g) return 3 * k + s;
  }
  return -1;
}

// ---------------------------------------------------------------------------------------
// second-order forward-mode arithmetic
// ---------------------------------------------------------------------------------------
static inline int hix(int a, int b) {  // upper-triangle index of (a,b)
  if (a > b) std::swap(a, b);
  static const int T[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  return T[a][b];
}
static HD hd_var(double v, int d) {
  HD r;
  r.v = v;
  r.g[d] = 1.0;
  return r;
}
static HD hd_const(double v) {
  HD r;
  r.v = v;
  return r;
}
static HD operator+(const HD& a, const HD& b) {
  HD r;
  r.v = a.v + b.v;
  for (int i = 0; i < 3; ++i) r.g[i] = a.g[i] + b.g[i];
  for (int i = 0; i < 6; ++i) r.h[i] = a.h[i] + b.h[i];
  return r;
}
static HD operator-(const HD& a, const HD& b) {
  HD r;
  r.v = a.v - b.v;
  for (int i = 0; i < 3; ++i) r.g[i] = a.g[i] - b.g[i];
  for (int i = 0; i < 6; ++i) r.h[i] = a.h[i] - b.h[i];
  return r;
}
static HD operator*(double s, const HD& a) {
  HD r;
  r.v = s * a.v;
  for (int i = 0; i < 3; ++i) r.g[i] = s * a.g[i];
  for (int i = 0; i < 6; ++i) r.h[i] = s * a.h[i];
  return r;
}
static HD operator*(const HD& a, const HD& b) {
  HD r;
  r.v = a.v * b.v;
  for (int i = 0; i < 3; ++i) r.g[i] = a.v * b.g[i] + b.v * a.g[i];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j)
      r.h[hix(i, j)] = a.v * b.h[hix(i, j)] + b.v * a.h[hix(i, j)] + a.g[i] * b.g[j] + a.g[j] * b.g[i];
  return r;
}
// unary chain rule: f(u) with f', f''
static HD chain(const HD& u, double f, double f1, double f2) {
  HD r;
  r.v = f;
  for (int i = 0; i < 3; ++i) r.g[i] = f1 * u.g[i];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) r.h[hix(i, j)] = f1 * u.h[hix(i, j)] + f2 * u.g[i] * u.g[j];
  return r;
}
static HD hsqrt(const HD& u) {
  double s = std::sqrt(u.v);
  return chain(u, s, 0.5 / s, -0.25 / (s * u.v));
}
static HD hsin(const HD& u) { return chain(u, std::sin(u.v), std::cos(u.v), -std::sin(u.v)); }
static HD hcos(const HD& u) { return chain(u, std::cos(u.v), -std::sin(u.v), -std::cos(u.v)); }
static HD hrecip(const HD& u) { return chain(u, 1.0 / u.v, -1.0 / (u.v * u.v), 2.0 / (u.v * u.v * u.v)); }
static HD hacos(const HD& u) {
  double q = 1.0 - u.v * u.v;
  double sq = std::sqrt(q);
  return chain(u, std::acos(u.v), -1.0 / sq, -u.v / (q * sq));
}
// atan2(y, x) with the binary chain rule
static HD hatan2(const HD& y, const HD& x) {
  double r2 = x.v * x.v + y.v * y.v;
  double fy = x.v / r2, fx = -y.v / r2;
  double fxx = 2 * x.v * y.v / (r2 * r2), fyy = -fxx, fxy = (y.v * y.v - x.v * x.v) / (r2 * r2);
  HD r;
  r.v = std::atan2(y.v, x.v);
  for (int i = 0; i < 3; ++i) r.g[i] = fx * x.g[i] + fy * y.g[i];
  for (int i = 0; i < 3; ++i)
    for (int j = i; j < 3; ++j) {
      int k = hix(i, j);
      r.h[k] = fx * x.h[k] + fy * y.h[k] + fxx * x.g[i] * x.g[j] + fyy * y.g[i] * y.g[j] +
               fxy * (x.g[i] * y.g[j] + y.g[i] * x.g[j]);
    }
  return r;
}

LevelSet::LevelSet(const kfbi_shape& shape) : s(shape) {
  const double* p = s.param;
  double half[3];
  switch (s.kind) {
    case KFBI_SPHERE: half[0] = half[1] = half[2] = p[0]; break;
    case KFBI_ELLIPSOID: {
      double a = std::max(p[0], std::max(p[1], p[2]));
      half[0] = half[1] = a;
      half[2] = p[2];
      break;
    }
    case KFBI_STAR: half[0] = half[1] = half[2] = p[0] + std::fabs(p[1]); break;
    case KFBI_TORUS: half[0] = half[1] = p[0] + p[1]; half[2] = p[0]; break;
    default: throw std::invalid_argument("unknown shape kind");
  }
  for (int d = 0; d < 3; ++d) {
    bb_lo[d] = s.center[d] - half[d];
    bb_hi[d] = s.center[d] + half[d];
  }
}

double LevelSet::value(double x, double y, double z) const {
  const double* p = s.param;
  x -= s.center[0];
  y -= s.center[1];
  z -= s.center[2];
  switch (s.kind) {
    case KFBI_SPHERE: return std::sqrt(x * x + y * y + z * z) - p[0];
    case KFBI_ELLIPSOID: {
      double t = s.rot_z_deg * M_PI / 180.0;
      double xr = std::cos(t) * x + std::sin(t) * y, yr = -std::sin(t) * x + std::cos(t) * y;
      return (xr / p[0]) * (xr / p[0]) + (yr / p[1]) * (yr / p[1]) + (z / p[2]) * (z / p[2]) - 1.0;
    }
    case KFBI_STAR: {
      double rho = std::sqrt(x * x + y * y + z * z);
      double th = std::acos(z / rho), ph = std::atan2(y, x);
      return rho - (p[0] + p[1] * std::sin(p[2] * th) * std::cos(p[3] * ph));
    }
    case KFBI_TORUS: {
      double q = std::sqrt(x * x + y * y) - p[1];
      return std::sqrt(q * q + z * z) - p[0];
    }
  }
  return 1.0;
}

HD LevelSet::eval(double x0, double y0, double z0) const {
  const double* p = s.param;
  HD x = hd_var(x0, 0) - hd_const(s.center[0]);
  HD y = hd_var(y0, 1) - hd_const(s.center[1]);
  HD z = hd_var(z0, 2) - hd_const(s.center[2]);
  switch (s.kind) {
    case KFBI_SPHERE: return hsqrt(x * x + y * y + z * z) - hd_const(p[0]);
    case KFBI_ELLIPSOID: {
      double t = s.rot_z_deg * M_PI / 180.0;
      HD xr = std::cos(t) * x + std::sin(t) * y;
      HD yr = (-std::sin(t)) * x + std::cos(t) * y;
      HD a = (1.0 / p[0]) * xr, b = (1.0 / p[1]) * yr, c = (1.0 / p[2]) * z;
      return a * a + b * b + c * c - hd_const(1.0);
    }
    case KFBI_STAR: {
      HD rho = hsqrt(x * x + y * y + z * z);
      HD th = hacos(z * hrecip(rho));
      HD ph = hatan2(y, x);
      return rho - (hd_const(p[0]) + p[1] * (hsin(p[2] * th) * hcos(p[3] * ph)));
    }
    case KFBI_TORUS: {
      HD q = hsqrt(x * x + y * y) - hd_const(p[1]);
      return hsqrt(q * q + z * z) - hd_const(p[0]);
    }
  }
  return HD();
}

// ---------------------------------------------------------------------------------------
// node sides
// ---------------------------------------------------------------------------------------
static double node_coord(const Setup& S, int g, int d, int64_t idx) {
  // face grid g: integer positions along g; half positions elsewhere (and on T^0)
  return (g == d) ? S.lo + idx * S.h : S.lo + (idx + 0.5) * S.h;
}

static void classify(const LevelSet& ls, Setup& S) {
  const int N = S.N;
  for (int g = 0; g < 4; ++g) {
    S.side[g].assign((size_t)S.M, 0);
    int lo_i[3], hi_i[3];
    for (int d = 0; d < 3; ++d) {
      lo_i[d] = N;
      hi_i[d] = -1;
      for (int a = 0; a < N; ++a) {
        double c = node_coord(S, g, d, a);
        if (c >= ls.bb_lo[d] - S.h && c <= ls.bb_hi[d] + S.h) {
          lo_i[d] = std::min(lo_i[d], a);
          hi_i[d] = std::max(hi_i[d], a);
        }
      }
    }
    if (hi_i[0] < 0 || hi_i[1] < 0 || hi_i[2] < 0) continue;
    uint8_t* sd = S.side[g].data();
#pragma omp parallel for collapse(2) schedule(static)
    for (int i = lo_i[0]; i <= hi_i[0]; ++i)
      for (int j = lo_i[1]; j <= hi_i[1]; ++j)
        for (int k = lo_i[2]; k <= hi_i[2]; ++k) {
          double x = node_coord(S, g, 0, i), y = node_coord(S, g, 1, j), z = node_coord(S, g, 2, k);
          sd[((int64_t)i * N + j) * N + k] = ls.inside(x, y, z) ? 1 : 0;
        }
  }
}

// ---------------------------------------------------------------------------------------
// crossings
// ---------------------------------------------------------------------------------------
struct Raw {
  int32_t f, a, b, j;
  double pos;
};

static void crossings(const LevelSet& ls, Setup& S) {
  const int N = S.N;
  const double h = S.h, lo = S.lo;
  std::vector<Raw> all;
  for (int f = 0; f < 9; ++f) {
    Family F = family(f);
    int ax[2], c = 0;
    for (int d = 0; d < 3; ++d)
      if (d != F.k) ax[c++] = d;
    // transverse index ranges (integer coordinate on axis g: 0..N; half: 0..N-1)
    std::vector<int> I[2];
    std::vector<double> C[2];
    for (int t = 0; t < 2; ++t) {
      int d = ax[t];
      int cnt = (d == F.g) ? N + 1 : N;
      for (int a = 0; a < cnt; ++a) {
        double cc = (d == F.g) ? lo + a * h : lo + (a + 0.5) * h;
        if (cc >= ls.bb_lo[d] - h && cc <= ls.bb_hi[d] + h) {
          I[t].push_back(a);
          C[t].push_back(cc);
        }
      }
    }
    int jlo = std::max(0, (int)std::floor((ls.bb_lo[F.k] - h - lo) / (0.5 * h)));
    int jhi = std::min(2 * N, (int)std::ceil((ls.bb_hi[F.k] + h - lo) / (0.5 * h)));
    const int64_t nl = (int64_t)I[0].size() * (int64_t)I[1].size();
    std::vector<std::vector<Raw>> per(nl);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t L = 0; L < nl; ++L) {
      int t0 = (int)(L / I[1].size()), t1i = (int)(L % I[1].size());
      double P[3];
      P[ax[0]] = C[0][t0];
      P[ax[1]] = C[1][t1i];
      bool prev = false;
      for (int j = jlo; j <= jhi; ++j) {
        P[F.k] = lo + j * (0.5 * h);
        bool in = ls.inside(P[0], P[1], P[2]);
        if (j > jlo && in != prev) {
          // bisection on [s_{j-1}, s_j]; keep side(a) = prev
          double a = lo + (j - 1) * (0.5 * h), b = lo + j * (0.5 * h);
          for (int it = 0; it < 200; ++it) {
            double m = 0.5 * (a + b);
            if (m == a || m == b) break;
            double Q[3] = {P[0], P[1], P[2]};
            Q[F.k] = m;
            bool im = ls.inside(Q[0], Q[1], Q[2]);
            if (im == prev)
              a = m;
            else
              b = m;
          }
          per[L].push_back({f, I[0][t0], I[1][t1i], j - 1, 0.5 * (a + b)});
        }
        prev = in;
      }
    }
    for (auto& v : per) all.insert(all.end(), v.begin(), v.end());
  }
  const int64_t T = (int64_t)all.size();
  S.T = T;
  S.fam.resize(T);
  S.l1.resize(T);
  S.l2.resize(T);
  S.jint.resize(T);
  S.pos.resize(T);
  S.xyz.resize(3 * T);
  for (int64_t t = 0; t < T; ++t) {
    const Raw& r = all[t];
    S.fam[t] = r.f;
    S.l1[t] = r.a;
    S.l2[t] = r.b;
    S.jint[t] = r.j;
    S.pos[t] = r.pos;
    Family F = family(r.f);
    int ax[2], c = 0;
    for (int d = 0; d < 3; ++d)
      if (d != F.k) ax[c++] = d;
    S.xyz[3 * t + F.k] = r.pos;
    int idx[2] = {r.a, r.b};
    for (int q = 0; q < 2; ++q) {
      int d = ax[q];
      S.xyz[3 * t + d] = (d == F.g) ? lo + idx[q] * h : lo + (idx[q] + 0.5) * h;
    }
  }
}

static void frames_and_control_points(const LevelSet& ls, Setup& S) {
  const int64_t T = S.T;
  S.nrm.resize(3 * T);
  S.t1.resize(3 * T);
  S.t2.resize(3 * T);
  S.kap.resize(4 * T);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < T; ++t) {
    HD p = ls.eval(S.xyz[3 * t], S.xyz[3 * t + 1], S.xyz[3 * t + 2]);
    double gn = std::sqrt(p.g[0] * p.g[0] + p.g[1] * p.g[1] + p.g[2] * p.g[2]);
    double n[3] = {p.g[0] / gn, p.g[1] / gn, p.g[2] / gn};
    int jm = 0;
    for (int d = 1; d < 3; ++d)
      if (std::fabs(n[d]) < std::fabs(n[jm])) jm = d;
    double e[3] = {0, 0, 0};
    e[jm] = 1.0;
    double a[3] = {e[1] * n[2] - e[2] * n[1], e[2] * n[0] - e[0] * n[2], e[0] * n[1] - e[1] * n[0]};
    double an = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    for (int d = 0; d < 3; ++d) a[d] /= an;
    double b[3] = {n[1] * a[2] - n[2] * a[1], n[2] * a[0] - n[0] * a[2], n[0] * a[1] - n[1] * a[0]};
    double H[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) H[i][j] = p.h[hix(i, j)];
    const double* tv[2] = {a, b};
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) {
        double s = 0;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) s += tv[u][i] * H[i][j] * tv[v][j];
        S.kap[4 * t + 2 * u + v] = -s / gn;
      }
    for (int d = 0; d < 3; ++d) {
      S.nrm[3 * t + d] = n[d];
      S.t1[3 * t + d] = a[d];
      S.t2[3 * t + d] = b[d];
    }
  }
  S.cp_of.assign(T, -1);
  S.cp_target.clear();
  for (int64_t t = 0; t < T; ++t) {
    Family F = family(S.fam[t]);
    if (F.g != GP) continue;
    const double* n = &S.nrm[3 * t];
    double mx = std::max(std::fabs(n[0]), std::max(std::fabs(n[1]), std::fabs(n[2])));
    if (std::fabs(n[F.k]) >= (1.0 - 1e-12) * mx) {
      S.cp_of[t] = (int64_t)S.cp_target.size();
      S.cp_target.push_back(t);
    }
  }
  S.n = (int64_t)S.cp_target.size();
}

void build_geometry(const kfbi_config& cfg, Setup& S) {
  LevelSet ls(cfg.shape);
  classify(ls, S);
  crossings(ls, S);
  frames_and_control_points(ls, S);
}

}  // namespace kfbi
