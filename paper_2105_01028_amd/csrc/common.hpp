// Host helpers shared by the medium and server halves of the C-ABI.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "device.hpp"
#include "host_setup.hpp"
#include "trinity.h"

namespace trinity {
// Message of the calling thread's last failed call.
inline std::string& last_error() {
  static thread_local std::string msg;
  return msg;
}

inline tr_status fail(tr_status s, const std::string& msg) {
  last_error() = msg;
  return s;
}

constexpr int kMaxDet = 64;

inline long long round_up(long long x, long long m) { return (x + m - 1) / m * m; }

inline bool valid_desc(const tr_grid_desc* d, std::string& err) {
  if (!d) return err = "null descriptor", false;
  if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->nx > 4096 || d->ny > 4096 || d->nz > 4096)
    return err = "grid sizes must be in 1..4096", false;
  // the collision kernels address five rows of the field with 32-bit byte
  // offsets: fewer than 2^31 / 20 voxels after padding to 256
  if (round_up((long long)d->nx * d->ny * d->nz, 256) * 20 >= (1LL << 31))
    return err = "grid too large: at most 107374080 voxels", false;
  if (!(d->dx_mm > 0) || !std::isfinite(d->dx_mm)) return err = "dx_mm must be > 0", false;
  if (d->nside < 1 || d->nside > 16) return err = "nside must be in 1..16", false;
  if (!(d->g > -1.0 && d->g < 1.0)) return err = "g must be in (-1, 1)", false;
  if (!(d->dt_ps >= 0) || !std::isfinite(d->dt_ps)) return err = "dt_ps must be >= 0", false;
  if (d->hg_norm != 0 && d->hg_norm != 1) return err = "bad hg_norm", false;
  if (d->coef != 0 && d->coef != 1) return err = "bad coef", false;
  if (d->advance < 0 || d->advance > 3) return err = "bad advance", false;
  if (d->advance == 3 && (d->precision != 0 || d->source != 0 || d->coef != 0 ||
                          ((d->nside_scatter == 0 || d->nside_scatter == d->nside) &&
                           12 * d->nside * d->nside > 192)))
    return err = "the retarded advance needs FP32, the explicit source, the paper's "
                 "coefficients, and at most 192 directions unless the source is on a "
                 "coarser angular grid", false;
  if (d->precision != 0 && d->precision != 1) return err = "bad precision", false;
  if (d->source != 0 && d->source != 1) return err = "bad source", false;
  if (d->transport != 0 && d->transport != 1) return err = "bad transport", false;
  if (d->retarded_source != 0 && d->retarded_source != 1)
    return err = "bad retarded_source", false;
  if (d->retarded_source == 1 && d->advance != 3)
    return err = "the flux-weighted source needs the retarded advance", false;
  if (d->nside_scatter != 0 && d->nside_scatter != d->nside) {
    const int ns = d->nside_scatter;
    if (ns < 1 || ns > d->nside || d->nside % ns != 0 || ((d->nside / ns) & (d->nside / ns - 1)))
      return err = "nside_scatter must divide nside by a power of two", false;
    if (12 * ns * ns > 192 || d->source != 0 || d->precision != 0)
      return err = "the two-level grid needs at most 192 scattering directions, the "
                   "explicit source and FP32", false;
  }
  if (d->source == 1 &&
      (d->hg_norm != 0 || d->coef != 0 || d->precision != 0 || 12 * d->nside * d->nside > 192))
    return err = "the implicit source needs the Sinkhorn phase matrix, the paper's "
                 "coefficients, FP32 and at most 192 directions", false;
  return true;
}

inline Field field_of(const tr_grid_desc* d) {
  Field f;
  f.ndir = 12 * d->nside * d->nside;
  f.NP = int(round_up(f.ndir, 32));
  f.nx = d->nx;
  f.ny = d->ny;
  f.nz = d->nz;
  f.V = d->nx * d->ny * d->nz;
  f.Vp = round_up(f.V, 256);
  return f;
}

inline unsigned short f32_to_bf16_bits(float x) {
  unsigned int u;
  std::memcpy(&u, &x, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
inline float bf16_bits_to_f32(unsigned short h) {
  unsigned int u = unsigned(h) << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

// Rounding P to fp32 leaves each column sum (the light scattered out of one
// incoming direction) off one by up to a few ulp of its largest entries, with a
// bias that creates or destroys light at every scattering.  Each pass moves the
// residual into the largest entry of the column that absorbs at least half of
// it, so that the relative change of any entry stays at the level of the
// rounding itself (a small entry, such as a backward-scattering one, would
// otherwise change by a large fraction of its value).
inline void conserve_columns_f32(std::vector<float>& P, int n, int ld) {
  std::vector<int> order(n);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int p, int q) {
      return P[size_t(p) * ld + j] > P[size_t(q) * ld + j];
    });
    for (int pass = 0; pass < 16; ++pass) {
      double s = 0;
      for (int i = 0; i < n; ++i) s += double(P[size_t(i) * ld + j]);
      const double r = 1.0 - s;
      if (r == 0.0) break;
      bool moved = false;
      for (int i : order) {
        float& p = P[size_t(i) * ld + j];
        const float np = float(double(p) + r);
        const double rn = r - (double(np) - double(p));
        if (np > 0.0f && std::fabs(rn) <= 0.5 * std::fabs(r)) {
          p = np;
          moved = true;
          break;
        }
      }
      if (!moved) break;
    }
  }
}

// The same for the bf16 pair P = P_hi + P_lo: nudge the low parts.
inline void conserve_columns_bf16(std::vector<uint16_t>& hi, std::vector<uint16_t>& lo, int n, int ld) {
  std::vector<int> order(n);
  auto val = [&](size_t k) { return double(bf16_bits_to_f32(hi[k])) + double(bf16_bits_to_f32(lo[k])); };
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int p, int q) {
      return val(size_t(p) * ld + j) > val(size_t(q) * ld + j);
    });
    for (int pass = 0; pass < 16; ++pass) {
      double s = 0;
      for (int i = 0; i < n; ++i) s += val(size_t(i) * ld + j);
      const double r = 1.0 - s;
      if (r == 0.0) break;
      bool moved = false;
      for (int i : order) {
        const size_t k = size_t(i) * ld + j;
        const double l = double(bf16_bits_to_f32(lo[k]));
        const uint16_t nl = f32_to_bf16_bits(float(l + r));
        const double rn = r - (double(bf16_bits_to_f32(nl)) - l);
        if (double(bf16_bits_to_f32(hi[k])) + double(bf16_bits_to_f32(nl)) > 0.0 &&
            std::fabs(rn) <= 0.5 * std::fabs(r)) {
          lo[k] = nl;
          moved = true;
          break;
        }
      }
      if (!moved) break;
    }
  }
}


// fp32 images of the discrete phase matrix: row-major P32 and its transpose
// PT, NP x NP with zero padding, columns summing to one (Sinkhorn form).
inline bool build_p32(const std::vector<Vec3>& dirs, double g, int hg_norm, int NP,
                      std::vector<float>& P32, std::vector<float>& PT) {
  std::vector<double> P64;
  if (!phase_matrix(dirs, g, hg_norm, P64)) return false;
  const int n = int(dirs.size());
  P32.assign(size_t(NP) * NP, 0.0f);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) P32[size_t(i) * NP + j] = float(P64[size_t(i) * n + j]);
  if (hg_norm == TR_HG_SINKHORN) conserve_columns_f32(P32, n, NP);
  PT.assign(P32.size(), 0.0f);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) PT[size_t(j) * NP + i] = P32[size_t(i) * NP + j];
  return true;
}

// Time bins of per-step detector records (Fig. 9 read-out): the light of step
// m is spread evenly over [m dt, (m+1) dt) and summed into bins of width bw.
// raw[k * stride + m], m < steps; out[k * nbins + j] (zeroed here).
inline void rebin(const double* raw, long long stride, long long steps, int ndet, double dt,
                  double bw, int nbins, double* out) {
  std::fill(out, out + size_t(ndet) * nbins, 0.0);
  for (long long m = 0; m < steps; ++m) {
    const double t0 = m * dt, t1 = (m + 1) * dt;
    const long long j0 = std::max(0LL, (long long)std::floor(t0 / bw));
    const long long j1 = std::min<long long>(nbins, (long long)std::ceil(t1 / bw));
    for (long long j = j0; j < j1; ++j) {
      const double lo = std::max(t0, j * bw), hi = std::min(t1, (j + 1) * bw);
      if (hi <= lo) continue;
      const double wgt = (hi - lo) / dt;
      for (int k = 0; k < ndet; ++k) out[size_t(k) * nbins + j] += raw[size_t(k) * stride + m] * wgt;
    }
  }
}

}  // namespace trinity
