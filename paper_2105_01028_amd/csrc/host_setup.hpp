// Host-side (FP64) set-up of a TRINITY medium: everything calculation Step 1
// of Sec. 2.4 fixes before the time loop.  No device code here.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace trinity {

constexpr double kC0 = 0.299792458;   // vacuum light speed, mm/ps

struct Vec3 {
  double x, y, z;
};

inline double dot(const Vec3& a, const Vec3& b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
inline double comp(const Vec3& a, int ax) { return ax == 0 ? a.x : (ax == 1 ? a.y : a.z); }

// HEALPix pixel centres, RING order (Sec. 2.1; Gorski et al. 2005).
std::vector<Vec3> healpix_ring(int nside);

// Discrete phase matrix P (row-major N x N) of Eq. (11)-(12): K_ij = p_HG(Omega_i .
// Omega_j) 4pi/N, then scaled to P = D K D with unit row and column sums
// (norm 0) or rows divided by their sums (norm 1).  Returns false if the
// scaling fails to converge.
bool phase_matrix(const std::vector<Vec3>& dirs, double g, int norm, std::vector<double>& P);

// Long-characteristic lattice (Sec. 2.1, Fig. 1): per direction the dominant
// axis a, the sign of Omega_a, the two transverse axes (b < c) and the ray's
// transverse offset R(k t) at plane k = 0..maxext for each transverse axis.
struct Lattice {
  int ndir = 0;
  int ext[3] = {0, 0, 0};   // voxels along x, y, z
  int maxext = 0;
  std::vector<int> axis, sign, bax, cax;
  std::vector<double> speed;       // |Omega_a|: planes per voxel of path
  std::vector<int> offset;         // [(d*2 + q)*(maxext+1) + k]
  int off(int d, int q, int k) const { return offset[(size_t(d) * 2 + q) * (maxext + 1) + k]; }
  // Next voxel along d's ray from voxel (x,y,z): returns its flat index, or -1 with
  // *face set to the face the ray leaves through.
  long long downwind(int d, int x, int y, int z, int* face) const;
};
Lattice build_lattice(const std::vector<Vec3>& dirs, int nx, int ny, int nz);

// Tables of phase advance with the moves in the collision kernel, from the
// lattice and its shift tables dl[(d * 2 + q) * dstride + k] (the shift along
// b (q = 0) or c (q = 1) into plane k, k = 1 .. maxext).  tab [(NP + 1) *
// maxext]: per direction d < ndir and coordinate p along its dominant axis,
// 64 times the flat offset of the move (shifts into the next plane, also past
// the last one) plus the mask of faces a voxel there may leave through (face
// 2 axis + side: the dominant-axis face always, the b / c face where the shift
// into the next plane is not zero); zero rows elsewhere.  dir [NP]:
// 10 axis | 3 << (2 axis + 8).  False, and the separate sweep is needed, when
// a direction's b or c shifts are not all -1, 0 or +1 of one sign.  reverse:
// the tables of the inverse moves (the adjoint's), each voxel back to where
// the forward ray came from, on the box taken periodically along the dominant
// axis: minus the shift into the voxel's own plane (into plane 0: minus the
// shift past the last plane), and the faces on the other side.
bool build_move_tables(const Lattice& lat, const std::vector<int8_t>& dl, int dstride, int NP,
                       std::vector<int>& tab, std::vector<int>& dir,
                       bool reverse = false);

// Time step (dt_ps > 0 wins; else dx * min(n) / c0) and per-voxel coefficients:
// a = e^{-mu_t l}, b from the coefficient form, r = min(n)/n_v.
struct Coefficients {
  double dt = 0, n_ref = 0, ell_ref = 0;
  bool uniform_n = true;
  std::vector<double> a, b, r;
};
bool build_coefficients(int nvox, const float* mua, const float* mus, const float* n, double dx,
                        double dt_ps, int coef, Coefficients& out, std::string& err);

// The pixel of the HEALPix grid of nside (numbered as healpix_ring) that
// contains the unit vector v.
int healpix_pixel(int nside, const Vec3& v);

// Parent (coarse pixel of nside_c) of every pixel of nside (a power-of-two multiple).
std::vector<int> healpix_parents(int nside, int nside_c);

// Eq. (9) weights of S0 and S1 for optical depth tau >= 0 (series below 0.1).
void eq9_weights(double tau, double& f0, double& f1);

// Eigen-decomposition of the symmetric n x n matrix A (row-major) by cyclic
// Jacobi rotations: A = V diag(lam) V^T, V[i*n + k] = component i of vector k.
void symmetric_eigen(const std::vector<double>& A, int n, std::vector<double>& V,
                     std::vector<double>& lam);

// Directions within cone_deg of axis (4 nearest when none), ascending index.
std::vector<int> cone_set(const std::vector<Vec3>& dirs, const Vec3& axis, double cone_deg);

// Photons of a Gaussian pulse (FWHM, centre t0) in step m, scaled so the pulse
// after t = 0 holds `total`.
double pulse_weight(long long m, double dt, double t0, double fwhm, double total);

// Fresnel reflectance, Eq. (14), light going from index n1 into n2 at incidence
// cosine cos1 (R = 1 at and beyond the critical angle).
double fresnel_R(double n1, double n2, double cos1);

// Interface crossings (Sec. 3.3): every (d, v) whose downwind voxel w has a
// different n, with the reflectance and the snapped reflected / refracted
// directions (-1 when totally reflected).
struct Interception {
  int d;
  long long v, w;
  double R;
  int d_refl, d_refr;
};
std::vector<Interception> interceptions(const Lattice& lat, const std::vector<Vec3>& dirs,
                                        const float* n);

}  // namespace trinity
