// Device-side argument blocks and launchers of the TRINITY step kernels.
// Shared by kernels.hip (definitions) and capi.cpp (callers).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace trinity {

// Per-direction lattice data on the device.
struct DevDir {
  int axis, sign, bax, cax;   // dominant axis a, sign of Omega_a, transverse axes b < c
  float nu;                   // planes advanced per step at the reference path (split mode)
  int unitb;                  // 1 if every plane-to-plane shift along b is -1, 0 or +1
  double nu64;                // same, FP64, for the phase-mode move rule
  // retarded stepping (below Courant one): a hop between planes takes
  // rD = rlag + rphi steps; rinvD = 1 / rD
  int rlag;
  float rphi, rD, rinvD;
};

// The photon field lives in N[d][v] buffers of NP rows (directions, padded to a
// multiple of 32 with zero rows) by Vp columns (voxels, padded to a multiple of
// 256 with zero columns).
struct Field {
  int ndir, NP;
  int V, nx, ny, nz;
  long long Vp;
};

struct InjectArgs {
  float* X;
  long long Vp;
  const int* pairs;        // [npairs][2] (direction, voxel)
  int npairs;
  const double* q;         // pulse weight per step
  int cap;                 // length of q and of the budget
  const int* step_ctr;
  double* budget;          // [cap][9]
  const DevDir* dirs;      // retarded stepping: a pair of direction d gets rD times its share
  int retarded;
  float* X2;               // two-level phase stepping: the field alternates between X (even
                           // steps) and X2 (odd steps); null otherwise
  // retarded stepping with a varying index (null otherwise): a pair (d, v) gets
  // rDc[d * 128 + class] times its share, class = mat[v] & 0x7f
  const uint8_t* mat;
  const float* rDc;
};

struct CollideArgs {
  const float* X;          // input field [NP][Vp]
  float* Y;                // output field [NP][Vp]
  const float* P;          // [NP][NP] fp32 phase matrix, transposed (zero padded)
  const float* Prow;       // [NP][NP] fp32 phase matrix, row-major (zero padded)
  const uint16_t* Phi;     // [NP][NP] bf16 high part (bf16-split mode)
  const uint16_t* Plo;     // [NP][NP] bf16 low part
  const float* a;          // [Vp]
  const float* b;          // [Vp]
  long long Vp;
  int NP;
  double* part;            // [2][nwg]: absorbed, total
  // implicit source (null otherwise): eigenvectors V[i][k] of P, row-major
  // [NP][NP], eigenvalues [NP], and per voxel w0 = omega f0, w1 = omega f1 and
  // the column-total factor c = (a + w0) / (1 - w1)
  const float* V;
  const float* lam;
  const float* w0;
  const float* w1;
  const float* cimp;
  // retarded stepping (null otherwise): history ring [H][NP][Vp] (slot = step
  // mod H), per voxel mu_t dx and omega, per direction row 1/|Omega_a| and 1/D
  // (zero on padding rows)
  float* ring;
  int H;
  const int* step_ctr;
  const float* mutdx;
  const float* omega;
  const float* hinvc;
  const float* hinvD;
  // phase moves in the collision's epilogue (launch_collide_move; null otherwise):
  // the field alternates between the two halves of pp ([2][NP][Vp]), step m
  // reads half m & 1 and writes the other.  mvtab[d][p] (NP + 1 rows of mvext
  // ints, row NP all zero for directions that stay) holds, for a voxel at
  // coordinate p along d's dominant axis, 64 times the flat offset of its move
  // (shifts into the next plane, also past the last one) plus a mask of the
  // faces it may leave through (face 2 axis + side, side 1 the high face);
  // mvdir[d] = 10 axis | 3 << (2 axis + 8) (the coordinate's shift in
  // a packed x | y << 10 | z << 20, and both faces of the dominant axis).
  // spart: [7][nwg] escape per face and light in the box.
  float* pp;
  const int* mvtab;
  const int* mvdir;
  const DevDir* dirs;
  int ndir, nx, ny, nz, nvox, mvext;
  int mvscramble;          // tile order multiplier, prime to the number of 256-voxel tiles
  int mvunscramble;        // its inverse modulo the number of tiles
  const unsigned* mvdet;   // bit per voxel column: a detector's voxel (light that leaves
                           // there is kept for the read-out; elsewhere it is only tallied)
  double* spart;
  // bf16-split with more than 192 directions (streamed P): [NP] column sums
  // sum_i P_lo[i][k], the column totals of the P_lo x_lo term the kernel drops
  const float* plocol;
  // retarded stepping: rvox = n_ref / n per voxel (null: uniform index), so a
  // hop from voxel v lasts D[d][v] = D_d / rvox[v] steps; with flux = 1 the
  // source is weighted by the scattered flux of each direction and hD holds D_d
  // per row (zero on padding rows)
  const float* rvox;
  const float* hD;
  int flux;
  // phase moves in the collision: 1 = read half 0 and write half 1 of pp
  // whatever the step's parity (the adjoint's recompute into its own slots)
  int mvfixed;
};

struct SweepArgs {
  const float* Y;          // post-collision field
  float* X;                // post-transport field
  long long Vp;
  int V, nx, ny, nz;
  const DevDir* dirs;
  const int8_t* delta;     // [d][2][dstride]: plane-to-plane transverse shift at plane k
  int dstride;
  const float* r;          // split mode: per-voxel path ratio
  const uint8_t* iface;    // Fresnel: 1 for voxels next to a different index
  const float* nvox;       // Fresnel: refractive index per voxel
  const int* islot;        // Fresnel: compact interface-voxel index
  float* icptF;            // Fresnel: intercepted flux [niface][ndir]
  int ndir;
  const int* step_ctr;
  double* part;            // [7][nwg]: escape per face 0..5, in the box
  const uint8_t* mat;      // split mode, optional: index class (bits 0-6), iface (bit 7)
  const float* rtab;       // split mode, with mat: path ratio per index class [128]
  const uint32_t* rowbits;  // split mode, with mat: bit of row (y, z) < kMaxRowBits set
                            // when all its voxels have class bgcls and none starts an
                            // interception
  unsigned bgcls;           // the class of most voxels
  const float* ring;        // retarded stepping: history ring [H][NP][Vp], slot = step mod H
  int H;
  long long slot;           // NP * Vp
  // two-level phase stepping (null otherwise): the sweep forms the collided
  // value a X + T[parent] share as it reads, from the field of this step's
  // parity (pp[m & 1]) into the other one; directions are taken in the order
  // dorder (the children of each coarse bin together)
  const float* tlT;
  const int* tlparent;
  const float* tla;
  float tlshare;
  float* pp0;
  float* pp1;
  const int* dorder;
  // retarded stepping with a varying index (launch_sweep_retarded_het): per
  // direction and index class ([NP][128]) the hop's whole steps, fraction and
  // 1/D; icptW[slot * ndir + d] = the content the intercepted light becomes
  // per unit of what reached the interface (reflected + refracted weights)
  const int* rlagc;
  const float* rphic;
  const float* rinvDc;
  const float* icptW;
  // two-level phase stepping, XCD-ordered grid (tlbpd a multiple of 8): a 1-D
  // grid of tlbpd x ndir workgroups; XCD x (workgroup ids x mod 8) takes row
  // blocks x, x + 8, ... of every direction, and the tlnk children of a coarse
  // bin one after another on the same block, so T[J]'s rows stay in its L2
  int tlbpd;
  int tlnk;
};

constexpr int kMaxRowBits = 65536;   // rows covered by the uniform-row bitmap (8 KB)

struct GatherArgs {
  float* X;
  long long Vp;
  const int* tgt_d;
  const int* tgt_v;
  const int* ptr;          // CSR over targets
  const int* src;          // slot into icptF
  const float* w;          // R (reflected share) or -R (refracted share F - R F)
  const float* icptF;
  int ntgt;
};

struct ReduceArgs {
  const double* cpart;
  int cnwg;
  const double* spart;
  int snwg;
  const float* Y;
  long long Vp;
  const int* det_pairs;    // [npairs][2] (detector, direction), grouped by detector
  const int* det_first;    // [ndet+1] start of each detector's pairs
  const int* det_vox;      // [ndet]
  int ndet;
  const DevDir* dirs;
  const float* r;
  int split;
  int* step_ctr;
  double* budget;          // [cap][9]
  double* det_steps;       // [ndet][cap]
  int cap;
  int* flag;               // bit 0: non-finite budget, bit 1: step beyond capacity
  double* scratch;         // [8] per-quantity sums of the current step
  int* done;               // workgroups finished (reset by the last one)
  const float* ring;       // retarded stepping: detectors read the history ring
  int H;
  long long slot;
  // two-level phase stepping: detectors read a X + T[parent] share from the
  // field of this step's parity
  const float* tlT;
  const int* tlparent;
  const float* tla;
  float tlshare;
  const float* pp0;
  const float* pp1;
  // phase moves in the collision (launch_collide_move): detectors read the
  // exiting light that the collision left in the field of this step's parity
  int mvfused;
  // retarded stepping with a varying index: class bytes and the per-class hop
  // tables of SweepArgs (detectors blend and scale by the voxel's class)
  const uint8_t* mat;
  const int* rlagc;
  const float* rphic;
  const float* rinvDc;
};

// One request of the batched server: its argument blocks as the single-medium
// kernels take them, plus what the batched kernels need to walk it.
struct ReqDev {
  InjectArgs inj;
  CollideArgs col;     // col.part: [2][ntiles] per-tile absorbed / total
  SweepArgs swp;       // swp.part: [7][ndir * bpd]
  ReduceArgs red;
  int nsteps;          // steps the request runs
  int ntiles;          // 256-voxel collide tiles
  int bpd;             // sweep blocks per direction
  int live;            // 1 while the slot holds a request
};

// Adjoint (transposed) step of phase mode, for one step m.
struct AdjArgs {
  const float* lam;        // adjoint of the field after the step, [NP][Vp]
  float* mu;               // adjoint of the post-collision field, [NP][Vp]
  float* lam_out;          // adjoint of the pre-collision field, [NP][Vp]
  const float* xs;         // forward pre-collision field of step m, [NP][Vp]
  const float* PT;         // P transposed, row-major [NP][NP] (what the forward calls Prow of P^T)
  const float* a;
  const float* b;
  double* ga;              // dL/da per voxel, accumulated
  double* gb;              // dL/db per voxel, accumulated
  long long Vp;
  int V, nx, ny, nz, ndir, NP;
  const DevDir* dirs;
  const int8_t* delta;
  int dstride;
  const int* det_pairs;    // [npairs][2] (detector, direction)
  int ndet_pairs;
  const int* det_vox;
  const double* seed;      // dL/d det[k][m], [ndet][steps]
  int steps;
};

// Two-level angular grid: fine field X, Y [ndir][Vp]; coarse sums M and
// coarse scattered light T [nc][Vp].
struct TwoLevelArgs {
  const float* X;
  float* Y;
  float* M;
  const float* T;
  const float* a;
  const float* b;
  const int* children;     // [nc][nkids] fine directions of each coarse bin
  const int* parent;       // [ndir]
  int ndir, nc, nkids;
  float share;             // 1 / nkids
  long long Vp;
  int V;
  double* part;            // [2][nwg] absorbed, total
  const float* X2;         // alternating field (see InjectArgs::X2), null otherwise
  const int* step_ctr;
  // retarded stepping (apply_hop): history ring [H][NP][Vp] (slot = step mod
  // H, NP * Vp floats each), per voxel mu_t dx and omega, per fine row
  // 1/|Omega_a| and 1/D
  float* ring;
  int H;
  long long slot;
  const float* mutdx;
  const float* omega;
  const float* hinvc;
  const float* hinvD;
  // retarded stepping with the flux-weighted source: the coarse sums weight
  // fine row i by (1 - a_i) / D_i and the hop collision takes D_i (hD[i]) times
  // the coarse source in place of 1 - a_i
  int flux;
  const float* hD;
};
long long coarse_sum_workgroups(const TwoLevelArgs& a);   // budget partial pairs written
hipError_t launch_coarse_sum(const TwoLevelArgs& a, hipStream_t s);
hipError_t launch_apply(const TwoLevelArgs& a, hipStream_t s);
// Retarded stepping on the two-level grid: the hop collision of every fine
// direction from the coarse source, into the history slot of the step; writes
// the budget partials (the layout of launch_coarse_sum, which it replaces).
hipError_t launch_apply_hop(const TwoLevelArgs& a, hipStream_t s);

// Launchers: queue the kernel on `s`.  Return the launch status.
hipError_t launch_inject(const InjectArgs& a, hipStream_t s);
hipError_t launch_collide(const CollideArgs& a, const Field& f, int bf16split, int nwg_cols,
                          hipStream_t s);
int collide_nwg(const Field& f, int bf16split);
// Implicit-source collision (A.V etc. set), NP <= 192, FP32.
// Retarded stepping below Courant one: collision with per-direction hop
// coefficients into the history ring, and the sweep that reads the ring at
// the retarded time.
hipError_t prepare_collide_hop(const Field& f);
hipError_t launch_collide_hop(const CollideArgs& a, const Field& f, hipStream_t s);
hipError_t launch_sweep_retarded(const SweepArgs& a, const Field& f, int blocks_per_dir,
                                 hipStream_t s);
// The same with a varying refractive index: per-voxel hop durations through
// index classes (a.mat, a.rlagc, a.rphic, a.rinvDc), hops across an index jump
// held in a.icptF for the gather (launch_gather with the content weights).
hipError_t launch_sweep_retarded_het(const SweepArgs& a, const Field& f, int blocks_per_dir,
                                     hipStream_t s);
// Two-level phase stepping: the sweep with the collided value formed as it reads.
hipError_t launch_sweep_twolevel(const SweepArgs& a, const Field& f, int blocks_per_dir,
                                 hipStream_t s);
hipError_t launch_collide_implicit(const CollideArgs& a, const Field& f, hipStream_t s);
// Phase stepping with the moves in the collision's epilogue (the A.pp fields
// set); needs use_collide_move(f).  Writes the collision partials to A.part
// ([2][nwg]) and the transport partials to A.spart ([7][nwg]), nwg =
// collide_nwg(f, bf16split).  With j.npairs > 0 it also does the step's
// injection (as launch_inject with j.X2 set), in place of launch_inject.
bool use_collide_move(const Field& f);
hipError_t prepare_collide_move(const Field& f, int bf16split);
hipError_t launch_collide_move(const CollideArgs& a, const InjectArgs& j, const Field& f,
                               int bf16split, hipStream_t s);
hipError_t prepare_collide_implicit(const Field& f);
hipError_t prepare_collide(const Field& f, int bf16split);   // once per process and shape
// fast_split_ok: nx is a multiple of 4 and every direction's b shifts are unit
// (then split mode with class bytes runs the fast kernel).
hipError_t launch_sweep(const SweepArgs& a, const Field& f, int split, int fresnel, int bpd,
                        hipStream_t s, int fast_split_ok = 0);
int sweep_blocks_per_dir(const Field& f, int retarded);
hipError_t launch_gather(const GatherArgs& a, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t s);
// Batched server step over `nslots` request slots: work lists citems (slot,
// tile) and sitems (slot, direction, block, 0), with counts[0] / counts[1]
// items, all in device memory so a captured graph stays valid as they change.
hipError_t launch_server_step(const ReqDev* reqs, int nslots, const int* citems,
                              const int* sitems, const int* counts, const float* Prow, int NP,
                              hipStream_t s);
hipError_t prepare_server(int NP);
// mu = T_m^T lam + D_m^T seed;  lam_out = a mu + b (P^T mu); ga += sum_d mu xs,
// gb += sum_d (P^T mu) xs.  Needs NP <= 192.
hipError_t launch_adjoint_step(const AdjArgs& a, int m, hipStream_t s);
hipError_t prepare_adjoint(int NP);
// Adjoint step m with the moves in the collision's epilogue (mv: the move
// arguments, pp the pair of mu halves, mvtab the reversed move tables, mvdet
// all zero), then the seeds of step m - 1 into the half it wrote.
hipError_t launch_adjoint_move_step(const AdjArgs& a, const CollideArgs& mv, int m,
                                    hipStream_t s);
hipError_t prepare_adjoint_move(int NP);
// The seeds of step m into a.mu.
hipError_t launch_adjoint_seeds(const AdjArgs& a, int m, hipStream_t s);
// Advance the device step counter by one (no tallies).
hipError_t launch_advance_step(int* ctr, hipStream_t s);
hipError_t launch_energy(const float* X, long long Vp, int ndir, int V, float* E, hipStream_t s);

// The allocation-free step's workspace: a file-scope device array of
// kScratchDoubles doubles (4 MiB) per GPU.  scratch_address gives its address
// on the current device (looked up once per device, with that device
// current); launch_zero_fill clears n doubles with a kernel (no memset node,
// so the call can sit under graph capture).
constexpr long long kScratchDoubles = 1LL << 19;
hipError_t scratch_address(double** out);
hipError_t launch_zero_fill(double* p, long long n, hipStream_t s);

}  // namespace trinity
