// Host set-up of a TRINITY medium in FP64.  See host_setup.hpp.
#include "host_setup.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace trinity {

namespace {
constexpr double kPi = 3.14159265358979323846;
constexpr double kAxisTie = 1e-12;   // |Omega| components this close count as tied
constexpr double kHalfEps = 1e-9;    // exact half offsets round toward zero
constexpr double kSnapTie = 1e-12;   // near-equal dot products snap to the lower index

// Nearest integer to x with halves rounded toward zero (an odd function).
int round_half_in(double x) {
  double m = std::floor(std::fabs(x) + 0.5 - kHalfEps);
  return int(x < 0 ? -m : m);
}

double hg(double mu, double g) {
  double den = 1.0 + g * g - 2.0 * g * mu;
  return (1.0 - g * g) / (4.0 * kPi * den * std::sqrt(den));
}

int nearest_dir(const std::vector<Vec3>& dirs, const Vec3& v) {
  double best = -1e300;
  for (const Vec3& o : dirs) best = std::max(best, dot(o, v));
  for (size_t i = 0; i < dirs.size(); ++i)
    if (dot(dirs[i], v) >= best - kSnapTie) return int(i);
  return 0;
}
}  // namespace

std::vector<Vec3> healpix_ring(int nside) {
  std::vector<Vec3> out;
  out.reserve(size_t(12) * nside * nside);
  const double ns = nside;
  for (int ring = 1; ring < 4 * nside; ++ring) {
    double z;
    int count;
    double dphi, shift;
    if (ring < nside) {                       // north polar cap
      z = 1.0 - double(ring) * ring / (3.0 * ns * ns);
      count = 4 * ring;
      dphi = kPi / (2.0 * ring);
      shift = 0.5;
    } else if (ring <= 3 * nside) {           // equatorial belt
      z = 4.0 / 3.0 - 2.0 * ring / (3.0 * ns);
      count = 4 * nside;
      dphi = kPi / (2.0 * ns);
      shift = ((ring - nside + 1) % 2) * 0.5;
    } else {                                  // south polar cap
      int k = 4 * nside - ring;
      z = -(1.0 - double(k) * k / (3.0 * ns * ns));
      count = 4 * k;
      dphi = kPi / (2.0 * k);
      shift = 0.5;
    }
    double s = std::sqrt((1.0 - z) * (1.0 + z));
    for (int j = 1; j <= count; ++j) {
      double phi = dphi * (j - shift);
      out.push_back({s * std::cos(phi), s * std::sin(phi), z});
    }
  }
  return out;
}

bool phase_matrix(const std::vector<Vec3>& dirs, double g, int norm, std::vector<double>& P) {
  const size_t n = dirs.size();
  const double w = 4.0 * kPi / double(n);
  P.assign(n * n, 0.0);
  for (size_t i = 0; i < n; ++i)
    for (size_t j = 0; j < n; ++j) {
      double c = std::min(1.0, std::max(-1.0, dot(dirs[i], dirs[j])));
      P[i * n + j] = w * hg(c, g);
    }
  if (norm == 1) {
    for (size_t i = 0; i < n; ++i) {
      double s = 0;
      for (size_t j = 0; j < n; ++j) s += P[i * n + j];
      for (size_t j = 0; j < n; ++j) P[i * n + j] /= s;
    }
    return true;
  }
  // Symmetric Sinkhorn-Knopp: find d > 0 with d_i (K d)_i = 1 by d <- sqrt(d / Kd).
  std::vector<double> d(n, 1.0), kd(n);
  bool done = false;
  for (int it = 0; it < 200000 && !done; ++it) {
    double worst = 0;
    for (size_t i = 0; i < n; ++i) {
      double s = 0;
      for (size_t j = 0; j < n; ++j) s += P[i * n + j] * d[j];
      kd[i] = s;
      worst = std::max(worst, std::fabs(d[i] * s - 1.0));
    }
    if (worst < 1e-14) {
      done = true;
      break;
    }
    for (size_t i = 0; i < n; ++i) d[i] = std::sqrt(d[i] / kd[i]);
  }
  if (!done) return false;
  for (size_t i = 0; i < n; ++i)
    for (size_t j = 0; j < n; ++j) P[i * n + j] = d[i] * P[i * n + j] * d[j];
  return true;
}

Lattice build_lattice(const std::vector<Vec3>& dirs, int nx, int ny, int nz) {
  Lattice L;
  L.ndir = int(dirs.size());
  L.ext[0] = nx;
  L.ext[1] = ny;
  L.ext[2] = nz;
  L.maxext = std::max(nx, std::max(ny, nz));
  const int nd = L.ndir;
  L.axis.resize(nd);
  L.sign.resize(nd);
  L.bax.resize(nd);
  L.cax.resize(nd);
  L.speed.resize(nd);
  L.offset.assign(size_t(nd) * 2 * (L.maxext + 1), 0);
  for (int d = 0; d < nd; ++d) {
    const Vec3& o = dirs[d];
    double mag[3] = {std::fabs(o.x), std::fabs(o.y), std::fabs(o.z)};
    double top = std::max(mag[0], std::max(mag[1], mag[2]));
    int a = mag[2] >= top - kAxisTie ? 2 : (mag[1] >= top - kAxisTie ? 1 : 0);
    int b = a == 0 ? 1 : 0;
    int c = a == 2 ? 1 : 2;
    L.axis[d] = a;
    L.bax[d] = b;
    L.cax[d] = c;
    L.sign[d] = comp(o, a) > 0 ? 1 : -1;
    L.speed[d] = mag[a];
    const double tb = comp(o, b) / mag[a], tc = comp(o, c) / mag[a];
    for (int k = 0; k <= L.maxext; ++k) {
      L.offset[(size_t(d) * 2 + 0) * (L.maxext + 1) + k] = round_half_in(k * tb);
      L.offset[(size_t(d) * 2 + 1) * (L.maxext + 1) + k] = round_half_in(k * tc);
    }
  }
  return L;
}

bool build_move_tables(const Lattice& lat, const std::vector<int8_t>& dl, int dstride, int NP,
                       std::vector<int>& tab, std::vector<int>& dir, bool reverse) {
  const int* ext = lat.ext;
  const long long st[3] = {1, ext[0], (long long)ext[0] * ext[1]};
  const int S = lat.maxext;
  tab.assign(size_t(NP + 1) * S, 0);
  dir.assign(size_t(NP), 0);
  auto shift = [&](int d, int q, int k) { return int(dl[(size_t(d) * 2 + q) * dstride + k]); };
  for (int d = 0; d < lat.ndir; ++d) {
    const int a = lat.axis[d], b = lat.bax[d], c = lat.cax[d], sg = lat.sign[d];
    // the b (c) shifts must be -1, 0 or +1 and of one sign along the ray
    int sb = 0, sc = 0;
    for (int k = 1; k <= ext[a]; ++k) {
      const int s0 = shift(d, 0, k), s1 = shift(d, 1, k);
      if (s0 < -1 || s0 > 1 || s1 < -1 || s1 > 1 || (s0 && sb && s0 != sb) ||
          (s1 && sc && s1 != sc))
        return false;
      if (s0) sb = s0;
      if (s1) sc = s1;
    }
    // reversed: the move back to the plane the ray came from, faces opposite
    const int rs = reverse ? -1 : 1;
    const int fa = 2 * a + (rs * sg > 0 ? 1 : 0), fb = 2 * b + (rs * sb > 0 ? 1 : 0),
              fc = 2 * c + (rs * sc > 0 ? 1 : 0);
    dir[d] = 10 * a | (3 << (2 * a)) << 8;
    for (int p = 0; p < ext[a]; ++p) {
      const int k = sg > 0 ? p : ext[a] - 1 - p;
      // forward: the shift into plane k + 1; reversed: minus the shift into
      // plane k (into plane 0 from past the last plane, the periodic box)
      const int ks = reverse ? (k >= 1 ? k : ext[a]) : k + 1;
      const int dbn = rs * shift(d, 0, ks), dcn = rs * shift(d, 1, ks);
      unsigned mk = 1u << fa;
      if (dbn) mk |= 1u << fb;
      if (dcn) mk |= 1u << fc;
      // |offset| <= 1 + 1023 + 1023^2 < 2^25: offset and mask share one int
      const long long off = rs * sg * st[a] + dbn * st[b] + dcn * st[c];
      tab[size_t(d) * S + p] = int(off * 64 + mk);
    }
  }
  return true;
}

long long Lattice::downwind(int d, int x, int y, int z, int* face) const {
  int p[3] = {x, y, z};
  const int a = axis[d], b = bax[d], c = cax[d], s = sign[d];
  const int k = s > 0 ? p[a] : ext[a] - 1 - p[a];
  *face = -1;
  if (k + 1 >= ext[a]) {
    *face = 2 * a + (s > 0 ? 1 : 0);
    return -1;
  }
  const int db = off(d, 0, k + 1) - off(d, 0, k);
  const int dc = off(d, 1, k + 1) - off(d, 1, k);
  int q[3];
  q[a] = p[a] + s;
  q[b] = p[b] + db;
  q[c] = p[c] + dc;
  if (q[b] < 0 || q[b] >= ext[b]) {
    *face = 2 * b + (db > 0 ? 1 : 0);
    return -1;
  }
  if (q[c] < 0 || q[c] >= ext[c]) {
    *face = 2 * c + (dc > 0 ? 1 : 0);
    return -1;
  }
  return (static_cast<long long>(q[2]) * ext[1] + q[1]) * ext[0] + q[0];
}

bool build_coefficients(int nvox, const float* mua, const float* mus, const float* n, double dx,
                        double dt_ps, int coef, Coefficients& out, std::string& err) {
  double nmin = 1e300, nmax = -1e300;
  for (int v = 0; v < nvox; ++v) {
    if (!(mua[v] >= 0.0f) || !(mus[v] >= 0.0f) || !std::isfinite(mua[v]) ||
        !std::isfinite(mus[v])) {
      err = "mu_a and mu_s must be finite and >= 0";
      return false;
    }
    if (!(n[v] >= 1.0f) || !std::isfinite(n[v])) {
      err = "refractive index must be finite and >= 1";
      return false;
    }
    nmin = std::min(nmin, double(n[v]));
    nmax = std::max(nmax, double(n[v]));
  }
  out.uniform_n = nmin == nmax;
  out.n_ref = nmin;
  out.dt = dt_ps > 0 ? dt_ps : dx * nmin / kC0;
  out.ell_ref = kC0 * out.dt / nmin;
  out.a.resize(nvox);
  out.b.resize(nvox);
  out.r.resize(nvox);
  for (int v = 0; v < nvox; ++v) {
    const double ell = kC0 * out.dt / double(n[v]);
    const double ma = mua[v], ms = mus[v], mt = ma + ms;
    const double a = std::exp(-mt * ell);
    double b;
    if (coef == 0)
      b = mt > 0 ? (ms / mt) * -std::expm1(-mt * ell) : 0.0;
    else
      b = std::exp(-ma * ell) * -std::expm1(-ms * ell);
    out.a[v] = a;
    out.b[v] = b;
    out.r[v] = nmin / double(n[v]);
  }
  return true;
}

int healpix_pixel(int nside, const Vec3& v) {
  const double z = std::max(-1.0, std::min(1.0, v.z));
  double phi = std::atan2(v.y, v.x);
  if (phi < 0) phi += 2.0 * kPi;
  double t = std::fmod(phi / (0.5 * kPi), 4.0);   // azimuth in quarter turns
  if (t < 0) t += 4.0;
  const int npix = 12 * nside * nside;
  if (std::fabs(z) <= 2.0 / 3.0) {
    // belt: pixels are bounded by the lines nside (t + 1/2) -/+ (3/4) nside z = const
    const double u = nside * (t + 0.5), w = 0.75 * nside * z;
    const long long up = (long long)std::floor(u - w);   // ascending boundary index
    const long long dn = (long long)std::floor(u + w);   // descending boundary index
    const int ring_b = int(nside + 1 + up - dn);           // 1 .. 2 nside + 1 from z = 2/3
    const int odd_start = (ring_b % 2 == 0) ? 1 : 0;      // rings whose first pixel is at azimuth 0
    long long in_ring = (up + dn - nside + odd_start + 1) / 2;
    in_ring = ((in_ring % (4 * nside)) + 4 * nside) % (4 * nside);
    // healpix_ring starts those rings one pixel later, at azimuth pi / (2 nside)
    if (odd_start) in_ring = (in_ring + 4 * nside - 1) % (4 * nside);
    return 2 * nside * (nside - 1) + (ring_b - 1) * 4 * nside + int(in_ring);
  }
  const double frac = t - std::floor(t);
  const double x = nside * std::sqrt(3.0 * (1.0 - std::fabs(z)));
  const int a = int(std::floor(frac * x)), b = int(std::floor((1.0 - frac) * x));
  const int ring = a + b + 1;                              // counted from the nearer pole
  const int in_ring = int(std::floor(t * ring)) % (4 * ring);
  return z > 0 ? 2 * ring * (ring - 1) + in_ring : npix - 2 * ring * (ring + 1) + in_ring;
}

std::vector<int> healpix_parents(int nside, int nside_c) {
  const std::vector<Vec3> d = healpix_ring(nside);
  std::vector<int> par(d.size());
  for (size_t i = 0; i < d.size(); ++i) par[i] = healpix_pixel(nside_c, d[i]);
  return par;
}

void eq9_weights(double tau, double& f0, double& f1) {
  if (tau >= 0.1) {
    f1 = (tau + std::expm1(-tau)) / tau;
  } else {
    // tau - 1 + e^-tau = sum_{k>=2} (-tau)^k / k!
    double term = tau / 2.0, sum = 0.0;
    for (int k = 2; k < 20; ++k) {
      sum += term;
      term *= -tau / double(k + 1);
    }
    f1 = sum;
  }
  f0 = -std::expm1(-tau) - f1;
}

void symmetric_eigen(const std::vector<double>& A0, int n, std::vector<double>& V,
                     std::vector<double>& lam) {
  std::vector<double> A(A0);
  V.assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) V[size_t(i) * n + i] = 1.0;
  auto at = [&](int i, int j) -> double& { return A[size_t(i) * n + j]; };
  double scale = 0.0;
  for (double x : A) scale = std::max(scale, std::fabs(x));
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += at(i, j) * at(i, j);
    if (std::sqrt(off) <= 1e-15 * scale * n) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = at(p, q);
        if (std::fabs(apq) <= 1e-300) continue;
        // rotation that zeroes A[p][q]
        const double theta = (at(q, q) - at(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = at(k, p), akq = at(k, q);
          at(k, p) = c * akp - s * akq;
          at(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = at(p, k), aqk = at(q, k);
          at(p, k) = c * apk - s * aqk;
          at(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double& vkp = V[size_t(k) * n + p];
          double& vkq = V[size_t(k) * n + q];
          const double x = vkp, y = vkq;
          vkp = c * x - s * y;
          vkq = s * x + c * y;
        }
      }
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = at(i, i);
}

std::vector<int> cone_set(const std::vector<Vec3>& dirs, const Vec3& axis, double cone_deg) {
  std::vector<int> in;
  const double cmin = std::cos(cone_deg * kPi / 180.0);
  for (size_t i = 0; i < dirs.size(); ++i)
    if (dot(dirs[i], axis) >= cmin) in.push_back(int(i));
  if (!in.empty()) return in;
  std::vector<int> idx(dirs.size());
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int p, int q) { return dot(dirs[p], axis) > dot(dirs[q], axis); });
  idx.resize(std::min<size_t>(4, idx.size()));
  std::sort(idx.begin(), idx.end());
  return idx;
}

double pulse_weight(long long m, double dt, double t0, double fwhm, double total) {
  const double sigma = fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
  auto cdf = [&](double t) { return 0.5 * (1.0 + std::erf((t - t0) / (sigma * std::sqrt(2.0)))); };
  const double tail = 1.0 - cdf(0.0);
  return (cdf(double(m + 1) * dt) - cdf(double(m) * dt)) / tail * total;
}

double fresnel_R(double n1, double n2, double cos1) {
  cos1 = std::min(1.0, std::max(0.0, cos1));
  const double sin1 = std::sqrt((1.0 - cos1) * (1.0 + cos1));
  const double sin2 = n1 / n2 * sin1;
  if (sin2 >= 1.0) return 1.0;
  if (sin1 < 1e-9) {
    const double r = (n1 - n2) / (n1 + n2);
    return r * r;
  }
  const double t1 = std::acos(cos1), t2 = std::asin(sin2);
  const double s_m = std::sin(t1 - t2), s_p = std::sin(t1 + t2);
  const double t_m = std::tan(t1 - t2), t_p = std::tan(t1 + t2);
  return 0.5 * ((s_m * s_m) / (s_p * s_p) + (t_m * t_m) / (t_p * t_p));
}

std::vector<Interception> interceptions(const Lattice& lat, const std::vector<Vec3>& dirs,
                                        const float* n) {
  const int nx = lat.ext[0], ny = lat.ext[1], nz = lat.ext[2];
  auto nat = [&](int x, int y, int z) {
    x = std::min(std::max(x, 0), nx - 1);
    y = std::min(std::max(y, 0), ny - 1);
    z = std::min(std::max(z, 0), nz - 1);
    return double(n[(size_t(z) * ny + y) * nx + x]);
  };
  std::vector<Interception> out;
  for (int d = 0; d < lat.ndir; ++d) {
    const Vec3& om = dirs[d];
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          int face;
          long long w = lat.downwind(d, x, y, z, &face);
          if (w < 0) continue;
          const long long v = (static_cast<long long>(z) * ny + y) * nx + x;
          const double n1 = n[v], n2 = n[w];
          if (n1 == n2) continue;
          Vec3 h{0.5 * (nat(x + 1, y, z) - nat(x - 1, y, z)),
                 0.5 * (nat(x, y + 1, z) - nat(x, y - 1, z)),
                 0.5 * (nat(x, y, z + 1) - nat(x, y, z - 1))};
          double hn = std::sqrt(dot(h, h));
          if (!(hn > 0.0)) {
            const int wx = int(w % nx), wy = int((w / nx) % ny), wz = int(w / (size_t(nx) * ny));
            h = Vec3{double(wx - x), double(wy - y), double(wz - z)};
            hn = std::sqrt(dot(h, h));
          }
          h = Vec3{h.x / hn, h.y / hn, h.z / hn};
          if (dot(om, h) < 0.0) h = Vec3{-h.x, -h.y, -h.z};
          const double c1 = dot(om, h);
          double R = fresnel_R(n1, n2, c1);
          const Vec3 refl{om.x - 2.0 * c1 * h.x, om.y - 2.0 * c1 * h.y, om.z - 2.0 * c1 * h.z};
          const int dr = nearest_dir(dirs, refl);
          const double eta = n1 / n2;
          const double s2sq = eta * eta * std::max(0.0, 1.0 - c1 * c1);
          int dtr = -1;
          if (s2sq >= 1.0) R = 1.0;
          if (R < 1.0) {
            const double k = std::sqrt(1.0 - s2sq) - eta * c1;
            const Vec3 t{eta * om.x + k * h.x, eta * om.y + k * h.y, eta * om.z + k * h.z};
            dtr = nearest_dir(dirs, t);
          }
          out.push_back({d, v, w, R, dr, dtr});
        }
  }
  return out;
}

}  // namespace trinity
