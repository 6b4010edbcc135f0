// Host FP64 Galerkin table of curl curl S for normalised voxel indicators.
//
// Section III-A of the paper: J is expanded in P_i = h^{-3/2} 1_{V_i} and tested
// with the same functions, giving N_ij = <N P_j, P_i> with N = curl curl S
// (Section III).  On a uniform grid the entry depends on m = i - j only.  Using
// curl curl = grad div - Laplacian and Laplacian S = -k^2 S - I, and the
// divergence theorem on both voxels for the grad-div part,
//
//   N^{ab}(m) = delta_ab (delta_{m0} + kappa^2 V(m)) - F^{ab}(m)        (h = 1)
//
//   V(m)      = int_{[-1,1]^3} G(m + s) prod_d (1 - |s_d|) ds
//   F^{aa}(m) = 2 g_a(m_a) - g_a(m_a + 1) - g_a(m_a - 1),
//   g_a(mu)   = int_{[-1,1]^2} G(mu e_a + m_perp + t) prod (1 - |t_d|) dt    (parallel faces)
//   F^{ab}(m) = int (1-|t|) [int_{m_a}^{m_a+1} - int_{m_a-1}^{m_a}] dDa
//                           [int_{m_b-1}^{m_b} - int_{m_b}^{m_b+1}] dDb  G(...)   (a != b)
//
// with G(R) = e^{i kappa R} / (4 pi R).  Every integral is a sum over unit
// lattice boxes with a polynomial weight; the origin (the only singular point)
// is a box vertex or at distance >= 1.  Vertex-singular boxes are mapped by a
// Duffy split into pyramids (the Jacobian cancels 1/R), the rest use tensor
// Gauss-Legendre whose order falls with the distance.  The table is computed
// once per plan, threaded over z-slices.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstring>
#include <thread>
#include <vector>

#include "vie_internal.hpp"

namespace vie {
namespace {

using cd = std::complex<double>;
constexpr double kPi = 3.14159265358979323846;

struct Rule {
  std::vector<double> x, w;   // nodes and weights on [0,1]
};

// Gauss-Legendre on [0,1]: roots of P_q by Newton iteration from Chebyshev
// guesses, in long double; weights 2/((1-t^2) P_q'(t)^2) mapped to [0,1].
Rule legendre_rule(int q) {
  Rule r;
  r.x.resize(q);
  r.w.resize(q);
  for (int i = 0; i < q; ++i) {
    long double t = std::cos(kPi * (i + 0.75L) / (q + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = t;
      for (int k = 2; k <= q; ++k) {
        long double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_q(t), p0 = P_{q-1}(t)
      dp = q * (t * p1 - p0) / (t * t - 1);
      long double dt = p1 / dp;
      t -= dt;
      if (std::fabs((double)dt) < 1e-19) break;
    }
    {
      long double p0 = 1, p1 = t;
      for (int k = 2; k <= q; ++k) {
        long double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (t * p1 - p0) / (t * t - 1);
    }
    r.x[i] = (double)(0.5L * (1 - t));
    r.w[i] = (double)(1.0L / ((1 - t * t) * dp * dp));
  }
  return r;
}

// Order for a non-singular unit box at squared distance d2 >= 1 from the origin.
// Chosen so that each box integral is accurate to ~1e-17 of 1/(4 pi d) for
// kappa <= 1.5 (the rate is that of the nearest complex singularity of 1/R).
int order_for(long d2) {
  if (d2 <= 1) return 15;
  if (d2 <= 2) return 13;
  if (d2 <= 4) return 12;
  if (d2 <= 9) return 11;
  if (d2 <= 16) return 10;
  if (d2 <= 36) return 9;
  if (d2 <= 100) return 8;
  if (d2 <= 400) return 7;
  if (d2 <= 2500) return 6;
  if (d2 <= 40000) return 5;
  return 4;
}

constexpr int kDuffyOrder = 18;

struct Rules {
  Rule r[32];
  Rules() {
    for (int q = 1; q < 32; ++q) r[q] = legendre_rule(q);
  }
};
const Rules& rules() {
  static Rules R;
  return R;
}

inline cd kernel(double x, double y, double z, double kappa) {
  double rr = std::sqrt(x * x + y * y + z * z);
  double s, c;
  sincos(kappa * rr, &s, &c);
  double f = 1.0 / (4 * kPi * rr);
  return cd(c * f, s * f);
}

// Weight of one axis on a unit box: al + be * t, t = x - lo in [0,1].
struct Lin {
  double al, be;
  double operator()(double t) const { return al + be * t; }
};

// int over the unit box [lo, lo+1]^3 of G(x) prod_d w_d(x_d - lo_d)
cd box3(const long lo[3], const Lin w[3], double kappa) {
  bool sing = true;
  long d2 = 0;
  for (int d = 0; d < 3; ++d) {
    long n = lo[d] > 0 ? lo[d] : (lo[d] + 1 < 0 ? -(lo[d] + 1) : 0);
    d2 += n * n;
    if (lo[d] != 0 && lo[d] != -1) sing = false;
  }
  cd acc = 0;
  if (!sing) {
    const Rule& R = rules().r[order_for(d2)];
    const int q = (int)R.x.size();
    for (int i = 0; i < q; ++i) {
      double xi = lo[0] + R.x[i], wi = R.w[i] * w[0](R.x[i]);
      for (int j = 0; j < q; ++j) {
        double yj = lo[1] + R.x[j], wj = wi * R.w[j] * w[1](R.x[j]);
        cd row = 0;
        for (int k = 0; k < q; ++k) {
          double zk = lo[2] + R.x[k];
          row += kernel(xi, yj, zk, kappa) * (R.w[k] * w[2](R.x[k]));
        }
        acc += row * wj;
      }
    }
    return acc;
  }
  // Vertex at the origin: x_d = sg_d * xi_d, xi in [0,1]^3, local t_d = x_d - lo_d.
  // Pyramid p (xi_p largest): xi_p = u, the other two u*v, u*w; Jacobian u^2.
  const Rule& R = rules().r[kDuffyOrder];
  const int q = (int)R.x.size();
  double sg[3];
  for (int d = 0; d < 3; ++d) sg[d] = lo[d] == 0 ? 1.0 : -1.0;
  for (int p = 0; p < 3; ++p) {
    int o1 = (p + 1) % 3, o2 = (p + 2) % 3;
    for (int i = 0; i < q; ++i) {
      double u = R.x[i], wu = R.w[i] * u * u;
      for (int j = 0; j < q; ++j) {
        double v = R.x[j];
        for (int k = 0; k < q; ++k) {
          double ww = R.x[k];
          double xi[3];
          xi[p] = u;
          xi[o1] = u * v;
          xi[o2] = u * ww;
          double x[3], wt = 1;
          for (int d = 0; d < 3; ++d) {
            x[d] = sg[d] * xi[d];
            wt *= w[d](x[d] - (double)lo[d]);
          }
          acc += kernel(x[0], x[1], x[2], kappa) * (wu * R.w[j] * R.w[k] * wt);
        }
      }
    }
  }
  return acc;
}

// int over the unit square [lo, lo+1]^2 in the plane x_a = mu of G(x) prod w
cd box2(int a, long mu, const long lo[2], const Lin w[2], double kappa) {
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  bool sing = (mu == 0);
  long d2 = mu * mu;
  for (int d = 0; d < 2; ++d) {
    long n = lo[d] > 0 ? lo[d] : (lo[d] + 1 < 0 ? -(lo[d] + 1) : 0);
    d2 += n * n;
    if (lo[d] != 0 && lo[d] != -1) sing = false;
  }
  cd acc = 0;
  double x[3];
  x[a] = (double)mu;
  if (!sing) {
    const Rule& R = rules().r[order_for(d2)];
    const int q = (int)R.x.size();
    for (int i = 0; i < q; ++i) {
      x[b] = lo[0] + R.x[i];
      double wi = R.w[i] * w[0](R.x[i]);
      for (int j = 0; j < q; ++j) {
        x[c] = lo[1] + R.x[j];
        acc += kernel(x[0], x[1], x[2], kappa) * (wi * R.w[j] * w[1](R.x[j]));
      }
    }
    return acc;
  }
  // Vertex at the origin; two triangles, xi_p = u, the other u*v, Jacobian u.
  const Rule& R = rules().r[kDuffyOrder];
  const int q = (int)R.x.size();
  double sg[2] = {lo[0] == 0 ? 1.0 : -1.0, lo[1] == 0 ? 1.0 : -1.0};
  for (int p = 0; p < 2; ++p) {
    for (int i = 0; i < q; ++i) {
      double u = R.x[i];
      for (int j = 0; j < q; ++j) {
        double xi[2];
        xi[p] = u;
        xi[1 - p] = u * R.x[j];
        double t0 = sg[0] * xi[0], t1 = sg[1] * xi[1];
        x[b] = t0;
        x[c] = t1;
        double wt = w[0](t0 - (double)lo[0]) * w[1](t1 - (double)lo[1]);
        acc += kernel(x[0], x[1], x[2], kappa) * (R.w[i] * u * R.w[j] * wt);
      }
    }
  }
  return acc;
}

// The tent (1 - |x - c|) on [c-1, c+1] as two unit pieces in local t.
inline void tent(long c, int side, long* lo, Lin* w) {
  if (side == 0) {
    *lo = c - 1;
    *w = Lin{0.0, 1.0};
  } else {
    *lo = c;
    *w = Lin{1.0, -1.0};
  }
}

cd volume_term(const long m[3], double kappa) {
  cd acc = 0;
  for (int s = 0; s < 8; ++s) {
    long lo[3];
    Lin w[3];
    for (int d = 0; d < 3; ++d) tent(m[d], (s >> d) & 1, &lo[d], &w[d]);
    acc += box3(lo, w, kappa);
  }
  return acc;
}

// g_a(mu, m_b, m_c) with (b, c) = the cyclic successors of a
cd face_parallel(int a, long mu, long mb, long mc, double kappa) {
  cd acc = 0;
  for (int s = 0; s < 4; ++s) {
    long lo[2];
    Lin w[2];
    tent(mb, s & 1, &lo[0], &w[0]);
    tent(mc, (s >> 1) & 1, &lo[1], &w[1]);
    acc += box2(a, mu, lo, w, kappa);
  }
  return acc;
}

cd face_orthogonal(int a, int b, const long m[3], double kappa) {
  const int c = 3 - a - b;
  cd acc = 0;
  for (int sa = 0; sa < 2; ++sa)
    for (int sb = 0; sb < 2; ++sb)
      for (int sc = 0; sc < 2; ++sc) {
        long lo[3];
        Lin w[3];
        lo[a] = sa == 0 ? m[a] : m[a] - 1;
        w[a] = Lin{sa == 0 ? 1.0 : -1.0, 0.0};
        lo[b] = sb == 0 ? m[b] - 1 : m[b];
        w[b] = Lin{sb == 0 ? 1.0 : -1.0, 0.0};
        tent(m[c], sc, &lo[c], &w[c]);
        acc += box3(lo, w, kappa);
      }
  return acc;
}

// Q_k(m) of the curl table: a signed unit step along k (+1 on [m_k, m_k+1],
// -1 on [m_k-1, m_k]) and the tent along the two other axes
cd curl_q(int k, const long m[3], double kappa) {
  const int p0 = (k + 1) % 3, p1 = (k + 2) % 3;
  cd acc = 0;
  for (int sk = 0; sk < 2; ++sk)
    for (int s0 = 0; s0 < 2; ++s0)
      for (int s1 = 0; s1 < 2; ++s1) {
        long lo[3];
        Lin w[3];
        lo[k] = sk == 0 ? m[k] : m[k] - 1;
        w[k] = Lin{sk == 0 ? 1.0 : -1.0, 0.0};
        tent(m[p0], s0, &lo[p0], &w[p0]);
        tent(m[p1], s1, &lo[p1], &w[p1]);
        acc += box3(lo, w, kappa);
      }
  return acc;
}

template <typename F>
void run_threads(int nthreads, long count, F&& body) {
  std::atomic<long> next{0};
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t)
    th.emplace_back([&] {
      for (;;) {
        long i = next.fetch_add(1);
        if (i >= count) break;
        body(i);
      }
    });
  for (auto& t : th) t.join();
}

}  // namespace

// Galerkin table of K = curl S (the magnetic-electric coupling of the JM-VIE,
// Section III): with Phi_j = int_{V_j} G and the divergence theorem on the
// testing voxel, K^{ab}(m) = eps_{akb} Q_k(m) (h = 1, k the axis other than a
// and b), Q_k(m) = int G(d) [1_{[m_k,m_k+1]} - 1_{[m_k-1,m_k]}](d_k)
// prod_{l != k} (1 - |d_l - m_l|) dd.  Output out[3][n1][n2][n3] for the
// components (0,1), (0,2), (1,2): -Q_2, +Q_1, -Q_0.  K^{ba} = -K^{ab}; Q_k is odd
// in m_k and even in the other offsets.
int curl_table(const int n[3], double kappa, std::complex<double>* out, int nthreads) {
  const long n1 = n[0], n2 = n[1], n3 = n[2];
  const long N = n1 * n2 * n3;
  (void)rules();
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  run_threads(nthreads, n1 * n2, [&](long row) {
    long m[3];
    m[0] = row / n2;
    m[1] = row % n2;
    for (m[2] = 0; m[2] < n3; ++m[2]) {
      const long idx = (m[0] * n2 + m[1]) * n3 + m[2];
      out[0 * N + idx] = -curl_q(2, m, kappa);
      out[1 * N + idx] = curl_q(1, m, kappa);
      out[2 * N + idx] = -curl_q(0, m, kappa);
    }
  });
  return 0;
}

int green_table(const int n[3], double kappa, std::complex<double>* out, int nthreads) {
  const long n1 = n[0], n2 = n[1], n3 = n[2];
  const long N = n1 * n2 * n3;
  (void)rules();
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  // g_a on mu in [0, n_a], m_b in [0, n_b), m_c in [0, n_c) (g is even in each argument)
  std::vector<cd> g[3];
  long gdim[3][3];
  for (int a = 0; a < 3; ++a) {
    int b = (a + 1) % 3, c = (a + 2) % 3;
    gdim[a][0] = n[a] + 1;
    gdim[a][1] = n[b];
    gdim[a][2] = n[c];
    g[a].resize(gdim[a][0] * gdim[a][1] * gdim[a][2]);
  }
  auto run = [&](auto&& body, long count) {
    std::atomic<long> next{0};
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t)
      th.emplace_back([&] {
        for (;;) {
          long i = next.fetch_add(1);
          if (i >= count) break;
          body(i);
        }
      });
    for (auto& t : th) t.join();
  };
  for (int a = 0; a < 3; ++a) {
    long d0 = gdim[a][0], d1 = gdim[a][1], d2 = gdim[a][2];
    run([&](long row) {
      long mu = row / d1, mb = row % d1;
      for (long mc = 0; mc < d2; ++mc)
        g[a][(mu * d1 + mb) * d2 + mc] = face_parallel(a, mu, mb, mc, kappa);
    }, d0 * d1);
  }
  auto gval = [&](int a, long mu, const long m[3]) -> cd {
    int b = (a + 1) % 3, c = (a + 2) % 3;
    long amu = mu < 0 ? -mu : mu;
    return g[a][(amu * gdim[a][1] + m[b]) * gdim[a][2] + m[c]];
  };
  run([&](long row) {   // one (m1, m2) column of m3 values
    long m[3];
    m[0] = row / n2;
    m[1] = row % n2;
    for (m[2] = 0; m[2] < n3; ++m[2]) {
      const long idx = (m[0] * n2 + m[1]) * n3 + m[2];
      cd V = volume_term(m, kappa);
      bool zero = m[0] == 0 && m[1] == 0 && m[2] == 0;
      cd diag_common = (zero ? 1.0 : 0.0) + kappa * kappa * V;
      cd Faa[3];
      for (int a = 0; a < 3; ++a)
        Faa[a] = 2.0 * gval(a, m[a], m) - gval(a, m[a] + 1, m) - gval(a, m[a] - 1, m);
      // component order xx, xy, xz, yy, yz, zz
      out[0 * N + idx] = diag_common - Faa[0];
      out[1 * N + idx] = -face_orthogonal(0, 1, m, kappa);
      out[2 * N + idx] = -face_orthogonal(0, 2, m, kappa);
      out[3 * N + idx] = diag_common - Faa[1];
      out[4 * N + idx] = -face_orthogonal(1, 2, m, kappa);
      out[5 * N + idx] = diag_common - Faa[2];
    }
  }, n1 * n2);
  return 0;
}

}  // namespace vie
