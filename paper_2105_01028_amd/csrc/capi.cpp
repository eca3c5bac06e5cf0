// C-ABI of the TRINITY step library (include/trinity.h): medium life cycle,
// host set-up upload, the step loop (with hipGraph replay of the per-step
// kernel sequence), read-out and rebinning.
#include "trinity.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "device.hpp"
#include "host_setup.hpp"

using namespace trinity;

constexpr int kGraphSteps = 16;   // steps per captured graph

struct tr_medium {
  tr_grid_desc desc{};
  hipStream_t stream = nullptr;
  Field f{};
  int mode = TR_ADVANCE_PHASE;
  bool fresnel = false;
  bool poisoned = false;
  double dt = 0;
  std::vector<Vec3> dirs;
  Lattice lat;
  Coefficients co;
  std::vector<float> nhost;
  std::vector<Interception> icpt;

  std::map<void*, size_t> owned;   // every device allocation and its size
  size_t bytes = 0;

  float *X = nullptr, *Y = nullptr, *P = nullptr, *Prow = nullptr, *a = nullptr, *b = nullptr,
        *r = nullptr;
  uint16_t *Phi = nullptr, *Plo = nullptr;
  float* plocol = nullptr;   // bf16-split: column sums of P_lo (the streamed kernels' fold)
  DevDir* ddirs = nullptr;
  int8_t* delta = nullptr;
  int dstride = 0;
  uint8_t* iface = nullptr;
  float* nvox = nullptr;
  int* islot = nullptr;
  float *V = nullptr, *lam = nullptr, *w0 = nullptr, *w1 = nullptr, *cimp = nullptr;  // implicit
  // retarded advance: history ring of H collided fields, per-voxel mu_t dx and
  // omega, per-row 1/|Omega_a| and 1/D
  float *ring = nullptr, *mutdx = nullptr, *omega = nullptr, *hinvc = nullptr, *hinvD = nullptr;
  int H = 0;
  // retarded advance with a varying index: hop tables per direction and index
  // class [NP][128] (whole steps, fraction, D, 1/D), D_d per row for the flux
  // source, and per interception the content the gather makes of it
  bool rhet = false;
  int* rlagc = nullptr;
  float *rphic = nullptr, *rDc = nullptr, *rinvDc = nullptr, *hD = nullptr, *icptW = nullptr;
  // two-level angular grid: coarse field of nc directions (NPc rows)
  bool twolevel = false;
  bool tlfused = false;     // two-level phase stepping: the sweep forms the collided value, the
                            // field alternates between X (even steps) and Y (odd steps)
  int nc = 0, NPc = 0, nkids = 0;
  // phase advance with the moves in the collision kernel (launch_collide_move):
  // the field alternates between X (even steps) and Y (odd steps); X and Y are
  // the two halves of one allocation
  bool mfused = false;
  int* mvtab = nullptr;
  int* mvdir = nullptr;
  int mvext = 0;
  int mvscramble = 1, mvunscramble = 1;
  unsigned* mvdet = nullptr;   // bit per voxel column: a detector's voxel
  float *M = nullptr, *T = nullptr, *zero = nullptr;
  int *children = nullptr, *parent = nullptr;
  double* cpart2 = nullptr;
  int cnwg2 = 0;
  uint8_t* mat = nullptr;   // split mode: index class | interface bit << 7, or null
  uint32_t* rowbits = nullptr;  // split mode: rows of background class only
  unsigned bgcls = 0;
  int fast_split = 0;       // nx % 4 == 0 and unit b shifts in every direction
  float* rtab = nullptr;    // split mode: path ratio of each index class
  float* icptF = nullptr;
  int niface = 0;
  int ntgt = 0;
  int *tgt_d = nullptr, *tgt_v = nullptr, *gptr = nullptr, *gsrc = nullptr;
  float* gw = nullptr;

  int* step_ctr = nullptr;
  int* flag = nullptr;
  double* rscratch = nullptr;
  int* rdone = nullptr;
  double *cpart = nullptr, *spart = nullptr;
  int cnwg = 0, snwg = 0, sweep_bpd = 0;
  double* scratch = nullptr;   // this device's allocation-free workspace (tr_step_noalloc)

  // capacity-dependent (reallocated when more steps are needed)
  int cap = 0;
  double* budget = nullptr;
  double* det_steps = nullptr;
  double* qdev = nullptr;

  // source
  bool have_source = false;
  int src_ix = 0, src_iy = 0, src_w = 1;
  double src_cone = 15, src_t0 = 20, src_fwhm = 10, src_total = 1;
  int npairs = 0;
  int* src_pairs = nullptr;

  // detectors
  int ndet = 0;
  std::vector<int> det_face, det_vox;
  double det_cone = 0;
  double bin_ps = 1.0;
  int nbins = 0;
  int* det_pairs = nullptr;
  int* det_first = nullptr;
  int* det_vox_dev = nullptr;

  long long steps_done = 0;

  hipGraphExec_t graph = nullptr;

  // checkpoints of tr_solve_checkpointed (one allocation of nckpt fields)
  float* ckpt = nullptr;
  int nckpt = 0, ckpt_every = 0;
  long long ckpt_steps = 0;
  std::vector<float> mua_host, mus_host;

  // kernel timing (tr_profile_begin / tr_profile_end)
  bool profiling = false;
  int prof_cap = 0, prof_used = 0;
  std::vector<hipEvent_t> prof_ev;   // [prof_cap][TR_K_COUNT][2]
  std::vector<int> prof_kind;        // kind of each recorded pair

  void free_events() {
    for (hipEvent_t e : prof_ev) (void)hipEventDestroy(e);
    prof_ev.clear();
    prof_kind.clear();
  }

  ~tr_medium() {
    free_events();
    if (graph) (void)hipGraphExecDestroy(graph);
    for (auto& kv : owned) (void)hipFree(kv.first);
  }

  template <class T>
  T* alloc(size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) return nullptr;
    owned[p] = count * sizeof(T);
    bytes += count * sizeof(T);
    return static_cast<T*>(p);
  }
  void release(void* p) {
    if (!p) return;
    auto it = owned.find(p);
    if (it == owned.end()) return;
    bytes -= it->second;
    owned.erase(it);
    (void)hipFree(p);
  }
  void drop_graph() {
    if (graph) (void)hipGraphExecDestroy(graph);
    graph = nullptr;
  }
};

namespace {

tr_status device_fail(tr_medium* m, hipError_t e, const char* what) {
  if (m) m->poisoned = true;
  return fail(TR_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define TR_CHECK_ALLOC(p) \
  if (!(p)) return fail(TR_ENOMEM, "device allocation failed")

// Bytes of the allocations that do not depend on the step capacity.
size_t fixed_bytes(const Field& f, int precision, int retarded, size_t niface_guess) {
  size_t b = 0;
  b += 2 * size_t(f.NP) * f.Vp * sizeof(float);         // X, Y
  b += 2 * size_t(f.NP) * f.NP * sizeof(float);          // P and its transpose
  if (precision == 1) b += 2 * size_t(f.NP) * f.NP * 2;  // P_hi, P_lo
  b += 3 * size_t(f.Vp) * sizeof(float);                 // a, b, r
  b += size_t(f.ndir) * sizeof(DevDir);
  b += size_t(f.ndir) * 2 * (std::max(f.nx, std::max(f.ny, f.nz)) + 2);
  const int cn = collide_nwg(f, precision), sn = sweep_blocks_per_dir(f, retarded) * f.ndir;
  b += (2 * size_t(cn) + 7 * size_t(std::max(sn, cn))) * sizeof(double);
  // move tables and detector bitmap of the phase moves in the collision
  const int S = std::max(f.nx, std::max(f.ny, f.nz));
  b += (size_t(f.NP + 1) * S * 2 + f.NP) * sizeof(int) + size_t(f.Vp / 32) * 4;
  b += niface_guess * f.ndir * sizeof(float);
  return b;
}

tr_status ensure_capacity(tr_medium* m, long long need) {
  if (need <= m->cap) return TR_OK;
  long long cap = std::max<long long>(need, std::max<long long>(1024, 2LL * m->cap));
  if (cap > (1LL << 30)) return fail(TR_EINVAL, "too many steps");
  hipError_t e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return device_fail(m, e, "synchronize");
  double* budget = m->alloc<double>(size_t(cap) * 9);
  double* dets = m->alloc<double>(size_t(std::max(m->ndet, 1)) * cap);
  double* q = m->alloc<double>(size_t(cap));
  if (!budget || !dets || !q) {
    m->release(budget);
    m->release(dets);
    m->release(q);
    return fail(TR_ENOMEM, "device allocation failed (step capacity)");
  }
  e = hipMemsetAsync(budget, 0, size_t(cap) * 9 * 8, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(dets, 0, size_t(std::max(m->ndet, 1)) * cap * 8, m->stream);
  if (e == hipSuccess && m->cap > 0) {
    e = hipMemcpyAsync(budget, m->budget, size_t(m->cap) * 9 * 8, hipMemcpyDeviceToDevice,
                       m->stream);
    for (int k = 0; k < m->ndet && e == hipSuccess; ++k)
      e = hipMemcpyAsync(dets + size_t(k) * cap, m->det_steps + size_t(k) * m->cap,
                         size_t(m->cap) * 8, hipMemcpyDeviceToDevice, m->stream);
  }
  std::vector<double> qh(cap, 0.0);
  if (m->have_source)
    for (long long s = 0; s < cap; ++s)
      qh[s] = pulse_weight(s, m->dt, m->src_t0, m->src_fwhm, m->src_total);
  if (e == hipSuccess) e = hipMemcpyAsync(q, qh.data(), size_t(cap) * 8, hipMemcpyHostToDevice, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return device_fail(m, e, "capacity growth");
  m->release(m->budget);
  m->release(m->det_steps);
  m->release(m->qdev);
  m->budget = budget;
  m->det_steps = dets;
  m->qdev = q;
  m->cap = int(cap);
  m->drop_graph();
  return TR_OK;
}

// The buffer that holds the field after the steps done so far: X, except in
// two-level phase stepping and with the moves in the collision, where the
// field alternates and odd steps end in Y.
float* state_field(tr_medium* m) {
  return (m->tlfused || m->mfused) && (m->steps_done & 1) ? m->Y : m->X;
}

// Event pair around one kernel while timing is active (no-op otherwise).
struct KernelTimer {
  tr_medium* m;
  int slot = -1;
  KernelTimer(tr_medium* mm, int kind) : m(mm) {
    if (!m->profiling || m->prof_used >= int(m->prof_kind.size())) return;
    slot = m->prof_used++;
    m->prof_kind[slot] = kind;
    (void)hipEventRecord(m->prof_ev[2 * slot], m->stream);
  }
  ~KernelTimer() {
    if (slot >= 0) (void)hipEventRecord(m->prof_ev[2 * slot + 1], m->stream);
  }
};

// Where a step's kernels keep their per-workgroup partial sums and the tally
// kernel its per-step sums and finished-workgroup counter: the medium's own
// buffers (tr_step), or the device's file-scope workspace (tr_step_noalloc).
struct Workspace {
  double* cpart;
  double* spart;
  double* cpart2;
  double* rscratch;
  int* rdone;
};

Workspace medium_workspace(tr_medium* m) {
  return Workspace{m->cpart, m->spart, m->cpart2, m->rscratch, m->rdone};
}

// The same pieces laid out in the device workspace; false if they do not fit.
// The counter takes the last double slot (it must start at zero).
bool scratch_workspace(tr_medium* m, Workspace* w, long long* used) {
  const long long nc = 2LL * m->cnwg, ns = 7LL * std::max(m->snwg, m->cnwg),
                  nc2 = m->twolevel ? 2LL * m->cnwg2 : 0LL;
  const long long need = nc + ns + nc2 + 8 + 1;
  *used = need;
  if (!m->scratch || need > kScratchDoubles) return false;
  double* p = m->scratch;
  w->cpart = p;
  w->spart = p + nc;
  w->cpart2 = m->twolevel ? p + nc + ns : nullptr;
  w->rscratch = p + nc + ns + nc2;
  w->rdone = reinterpret_cast<int*>(p + nc + ns + nc2 + 8);
  return true;
}

hipError_t queue_step(tr_medium* m, const Workspace& w) {
  const Field& f = m->f;
  hipError_t e;
  InjectArgs ia{m->X,   f.Vp,        m->src_pairs, m->npairs, m->qdev,
                m->cap, m->step_ctr, m->budget,    m->ddirs,  m->ring != nullptr,
                m->tlfused || m->mfused ? m->Y : nullptr};
  if (m->rhet) {
    ia.mat = m->mat;
    ia.rDc = m->rDc;
  }
  if (m->npairs > 0 && !m->mfused) {   // the collision with the moves injects itself
    KernelTimer t(m, TR_K_INJECT);
    if ((e = launch_inject(ia, m->stream)) != hipSuccess) return e;
  }
  if (m->twolevel) {
    TwoLevelArgs ta{m->X,     m->Y,          m->M,                   m->T,  m->a,
                    m->b,     m->children,   m->parent,              f.ndir, m->nc,
                    m->nkids, 1.0f / float(m->nkids), f.Vp,          f.V,   w.cpart,
                    m->tlfused ? m->Y : nullptr, m->step_ctr};
    if (m->ring) {
      ta.ring = m->ring;
      ta.H = m->H;
      ta.slot = (long long)f.NP * f.Vp;
      ta.mutdx = m->mutdx;
      ta.omega = m->omega;
      ta.hinvc = m->hinvc;
      ta.hinvD = m->hinvD;
      ta.hD = m->hD;
      ta.flux = m->desc.retarded_source;
    }
    Field fc = f;
    fc.ndir = m->nc;
    fc.NP = m->NPc;
    // coarse source T = b (P_c M); with the retarded history the factor is
    // omega, and each fine direction's (1 - a) comes in apply_hop
    CollideArgs cc{m->M, m->T, m->P, m->Prow, nullptr, nullptr, m->zero,
                   m->ring ? m->omega : m->b, f.Vp, m->NPc, w.cpart2};
    {
      KernelTimer t(m, TR_K_COARSE_SUM);
      if ((e = launch_coarse_sum(ta, m->stream)) != hipSuccess) return e;
    }
    {
      KernelTimer t(m, TR_K_COLLIDE);
      if ((e = launch_collide(cc, fc, 0, 0, m->stream)) != hipSuccess) return e;
    }
    if (m->ring) {
      KernelTimer t(m, TR_K_APPLY);
      if ((e = launch_apply_hop(ta, m->stream)) != hipSuccess) return e;
    } else if (!m->tlfused) {
      KernelTimer t(m, TR_K_APPLY);
      if ((e = launch_apply(ta, m->stream)) != hipSuccess) return e;
    }
  } else if (m->ring) {
    KernelTimer t(m, TR_K_COLLIDE);
    CollideArgs ca{};
    ca.X = m->X;
    ca.Prow = m->Prow;
    ca.Vp = f.Vp;
    ca.NP = f.NP;
    ca.part = w.cpart;
    ca.ring = m->ring;
    ca.H = m->H;
    ca.step_ctr = m->step_ctr;
    ca.mutdx = m->mutdx;
    ca.omega = m->omega;
    ca.hinvc = m->hinvc;
    ca.hinvD = m->hinvD;
    ca.rvox = m->rhet ? m->r : nullptr;
    ca.hD = m->hD;
    ca.flux = m->desc.retarded_source;
    if ((e = launch_collide_hop(ca, f, m->stream)) != hipSuccess) return e;
  } else if (m->mfused) {
    KernelTimer t(m, TR_K_COLLIDE);
    CollideArgs ca{};
    ca.Prow = m->Prow;
    ca.Phi = m->Phi;
    ca.Plo = m->Plo;
    ca.a = m->a;
    ca.b = m->b;
    ca.Vp = f.Vp;
    ca.NP = f.NP;
    ca.part = w.cpart;
    ca.step_ctr = m->step_ctr;
    ca.pp = m->X;
    ca.mvtab = m->mvtab;
    ca.mvdir = m->mvdir;
    ca.dirs = m->ddirs;
    ca.ndir = f.ndir;
    ca.nx = f.nx;
    ca.ny = f.ny;
    ca.nz = f.nz;
    ca.nvox = f.V;
    ca.mvext = m->mvext;
    ca.mvscramble = m->mvscramble;
    ca.mvdet = m->mvdet;
    ca.spart = w.spart;
    ca.mvunscramble = m->mvunscramble;
    if ((e = launch_collide_move(ca, ia, f, m->desc.precision, m->stream)) != hipSuccess) return e;
  } else {
    KernelTimer t(m, TR_K_COLLIDE);
    CollideArgs ca{m->X,   m->Y, m->P,  m->Prow, m->Phi, m->Plo, m->a,   m->b,
                   f.Vp,   f.NP, w.cpart, m->V, m->lam, m->w0,  m->w1, m->cimp};
    ca.plocol = m->plocol;
    e = m->V ? launch_collide_implicit(ca, f, m->stream)
             : launch_collide(ca, f, m->desc.precision, 0, m->stream);
    if (e != hipSuccess) return e;
  }
  const bool split = m->mode == TR_ADVANCE_SPLIT;
  if (!m->mfused) {
    KernelTimer t(m, TR_K_SWEEP);
    SweepArgs sa{m->Y, m->X, f.Vp, f.V, f.nx, f.ny, f.nz, m->ddirs, m->delta, m->dstride,
                 m->r, m->iface, m->nvox, m->islot, m->icptF, f.ndir, m->step_ctr, w.spart,
                 m->mat, m->rtab, m->rowbits, m->bgcls, m->ring, m->H, (long long)f.NP * f.Vp};
    if (m->tlfused) {
      sa.tlT = m->T;
      sa.tlparent = m->parent;
      sa.tla = m->a;
      sa.tlshare = 1.0f / float(m->nkids);
      sa.pp0 = m->X;
      sa.pp1 = m->Y;
      sa.dorder = m->children;   // the children of each coarse bin together
      if (m->sweep_bpd % 8 == 0) {
        sa.tlbpd = m->sweep_bpd;
        sa.tlnk = m->nkids;
      }
      e = launch_sweep_twolevel(sa, f, m->sweep_bpd, m->stream);
    } else if (m->ring && m->rhet) {
      sa.rlagc = m->rlagc;
      sa.rphic = m->rphic;
      sa.rinvDc = m->rinvDc;
      sa.icptW = m->icptW;
      e = launch_sweep_retarded_het(sa, f, m->sweep_bpd, m->stream);
    } else if (m->ring) {
      e = launch_sweep_retarded(sa, f, m->sweep_bpd, m->stream);
    } else {
      e = launch_sweep(sa, f, split, m->fresnel, m->sweep_bpd, m->stream, m->fast_split);
    }
    if (e != hipSuccess) return e;
  }
  if (m->fresnel) {
    KernelTimer t(m, TR_K_GATHER);
    GatherArgs ga{m->X, f.Vp, m->tgt_d, m->tgt_v, m->gptr, m->gsrc, m->gw, m->icptF, m->ntgt};
    if ((e = launch_gather(ga, m->stream)) != hipSuccess) return e;
  }
  KernelTimer t(m, TR_K_REDUCE);
  ReduceArgs ra{w.cpart, m->cnwg, w.spart, m->snwg, m->Y, f.Vp, m->det_pairs, m->det_first,
                m->det_vox_dev, m->ndet, m->ddirs, m->r, split ? 1 : 0, m->step_ctr, m->budget,
                m->det_steps, m->cap, m->flag, w.rscratch, w.rdone,
                m->ring, m->H, (long long)f.NP * f.Vp};
  if (m->tlfused) {
    ra.tlT = m->T;
    ra.tlparent = m->parent;
    ra.tla = m->a;
    ra.tlshare = 1.0f / float(m->nkids);
    ra.pp0 = m->X;
    ra.pp1 = m->Y;
  }
  if (m->rhet) {
    ra.mat = m->mat;
    ra.rlagc = m->rlagc;
    ra.rphic = m->rphic;
    ra.rinvDc = m->rinvDc;
  }
  if (m->mfused) {
    ra.snwg = m->cnwg;   // the transport partials come from the collision's workgroups
    ra.mvfused = 1;
    ra.pp0 = m->X;
    ra.pp1 = m->Y;
  }
  return launch_reduce(ra, m->stream);
}

// Detector (direction) pairs: accepted directions whose ray leaves the box
// through the detector's face from the detector's voxel.
tr_status upload_detector_pairs(tr_medium* m, const std::vector<std::vector<int>>& acc) {
  std::vector<int> pairs, first(1, 0);
  const int nx = m->f.nx, ny = m->f.ny;
  for (int k = 0; k < m->ndet; ++k) {
    const int v = m->det_vox[k];
    const int x = v % nx, y = (v / nx) % ny, z = v / (nx * ny);
    for (int d : acc[k]) {
      int face;
      if (m->lat.downwind(d, x, y, z, &face) < 0 && face == m->det_face[k]) {
        pairs.push_back(k);
        pairs.push_back(d);
      }
    }
    first.push_back(int(pairs.size() / 2));
  }
  int* dp = m->alloc<int>(std::max<size_t>(pairs.size(), 2));
  int* df = m->alloc<int>(first.size());
  int* dv = m->alloc<int>(std::max(m->ndet, 1));
  if (!dp || !df || !dv) return fail(TR_ENOMEM, "device allocation failed");
  hipError_t e = hipMemcpy(dp, pairs.data(), pairs.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(df, first.data(), first.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dv, m->det_vox.data(), m->ndet * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess && m->mvdet) {
    std::vector<unsigned> bits(size_t(m->f.Vp / 32), 0u);
    for (int v : m->det_vox) bits[size_t(v) >> 5] |= 1u << (v & 31);
    e = hipMemcpy(m->mvdet, bits.data(), bits.size() * 4, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return device_fail(m, e, "detector upload");
  m->det_pairs = dp;
  m->det_first = df;
  m->det_vox_dev = dv;
  return TR_OK;
}

tr_status check_medium(tr_medium* m) {
  if (!m) return fail(TR_EINVAL, "null medium");
  if (m->poisoned) return fail(TR_ESTATE, "medium is poisoned by an earlier device error");
  return TR_OK;
}

// Device bytes of a medium that do not depend on n: fields, tables, partials,
// the records of max_steps steps.
size_t base_bytes(const tr_grid_desc* desc, int ndet, int max_steps) {
  Field f = field_of(desc);
  size_t b = fixed_bytes(f, desc->precision, desc->advance == TR_ADVANCE_RETARDED, 0);
  if (desc->precision == TR_PREC_BF16SPLIT) b += size_t(f.NP) * sizeof(float);   // P_lo sums
  if (desc->source == TR_SOURCE_IMPLICIT)   // V, its eigenvalues, w0, w1, c
    b += (size_t(f.NP) * f.NP + f.NP + 3 * size_t(f.Vp)) * sizeof(float);
  if (desc->nside_scatter != 0 && desc->nside_scatter != desc->nside) {
    // coarse fields M and T, a zero row, children and parents, partials
    const long long NPc = round_up(12LL * desc->nside_scatter * desc->nside_scatter, 32);
    b += (2 * size_t(NPc) + 1) * f.Vp * sizeof(float) + 2 * size_t(f.ndir) * sizeof(int);
    b += 4 * (size_t(f.Vp / 256) + 64) * 16 * sizeof(double);
  }
  long long cap = std::max(1024, max_steps);
  b += size_t(cap) * (9 + std::max(ndet, 1) + 1) * sizeof(double);
  b += size_t(f.ndir) * 8 * sizeof(int) + 4096;
  return b;
}

// Header of a saved state (tr_save_state): the body follows it.
struct SavedState {
  char magic[8];
  uint64_t fingerprint;
  long long steps, ndir, nvox, ndet, history, total;
};
constexpr char kStateMagic[8] = {'T', 'R', 'S', 'T', 'A', 'T', 'E', '1'};

// FNV-1a, 64 bit, over bytes (the fingerprint of a saved state's medium).
struct Fnv1a {
  uint64_t h = 14695981039346656037ull;
  void bytes(const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  }
  template <class T> void val(T v) { bytes(&v, sizeof v); }
};

// What a saved state is only valid for: the resolved description, the
// medium arrays, the source and the detectors.
uint64_t state_fingerprint(const tr_medium* m) {
  Fnv1a h;
  const tr_grid_desc& d = m->desc;
  for (int v : {d.nx, d.ny, d.nz, d.nside, d.hg_norm, d.coef, m->mode, d.precision, d.source,
                d.nside_scatter, d.transport, d.retarded_source})
    h.val(v);
  for (double v : {d.dx_mm, d.g, m->dt}) h.val(v);
  h.bytes(m->mua_host.data(), m->mua_host.size() * sizeof(float));
  h.bytes(m->mus_host.data(), m->mus_host.size() * sizeof(float));
  h.bytes(m->nhost.data(), m->nhost.size() * sizeof(float));
  h.val(int(m->have_source));
  for (int v : {m->src_ix, m->src_iy, m->src_w}) h.val(v);
  for (double v : {m->src_cone, m->src_t0, m->src_fwhm, m->src_total}) h.val(v);
  h.val(m->ndet);
  h.bytes(m->det_face.data(), m->det_face.size() * sizeof(int));
  h.bytes(m->det_vox.data(), m->det_vox.size() * sizeof(int));
  for (double v : {m->det_cone, m->bin_ps}) h.val(v);
  h.val(m->nbins);
  return h.h;
}

size_t state_bytes(const tr_medium* m, long long steps) {
  return sizeof(SavedState) + size_t(1 + m->H) * m->f.ndir * m->f.V * sizeof(float) +
         size_t(steps) * (9 + m->ndet) * sizeof(double);
}

// The adjoint passes of tr_backward: dL/da and dL/db per voxel into hga, hgb
// (seed[k * steps + s] = dL/d det[k][s]).  The medium's field, step counter
// and records are left as they were.

// With the separate transposed sweep (media stepped with the sweep kernel):
// per segment, recompute its pre-collision fields from the checkpoint
// (inject, collide, sweep, tallies), then step backwards: transposed sweep,
// seeds, transposed collision.
tr_status backward_sweep(tr_medium* m, const std::vector<double>& seed, std::vector<double>& hga,
                         std::vector<double>& hgb) {
  const Field& f = m->f;
  const size_t NV = size_t(f.NP) * f.Vp;
  const long long steps = m->steps_done;
  const int K = m->ckpt_every;
  hipError_t e = prepare_adjoint(f.NP);
  if (e != hipSuccess) return device_fail(m, e, "adjoint set-up");
  float* lam = m->alloc<float>(NV);
  float* mu = m->alloc<float>(NV);
  float* seg = m->alloc<float>(NV * size_t(K));
  float* keep = m->alloc<float>(NV);
  double* ga = m->alloc<double>(f.Vp);
  double* gb = m->alloc<double>(f.Vp);
  double* sd = m->alloc<double>(seed.size());
  auto cleanup = [&]() {
    for (void* p : {(void*)lam, (void*)mu, (void*)seg, (void*)keep, (void*)ga, (void*)gb, (void*)sd})
      m->release(p);
  };
  if (!lam || !mu || !seg || !keep || !ga || !gb || !sd) {
    cleanup();
    return fail(TR_ENOMEM, "no device memory for the adjoint");
  }
  e = hipMemcpyAsync(keep, state_field(m), NV * 4, hipMemcpyDeviceToDevice, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(lam, 0, NV * 4, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(mu, 0, NV * 4, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(seg, 0, NV * 4 * size_t(K), m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(ga, 0, f.Vp * 8, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(gb, 0, f.Vp * 8, m->stream);
  if (e == hipSuccess) e = hipMemcpy(sd, seed.data(), seed.size() * 8, hipMemcpyHostToDevice);
  AdjArgs A{lam, mu, lam, nullptr, m->P, m->a, m->b, ga, gb, f.Vp, f.V, f.nx, f.ny, f.nz, f.ndir,
            f.NP, m->ddirs, m->delta, m->dstride, nullptr, 0, m->det_vox_dev, sd, int(steps)};
  // detector pairs of the medium (host copy rebuilt from the device lists)
  std::vector<int> first(m->ndet + 1);
  if (e == hipSuccess) e = hipMemcpy(first.data(), m->det_first, first.size() * 4, hipMemcpyDeviceToHost);
  A.det_pairs = m->det_pairs;
  A.ndet_pairs = first[m->ndet];
  const bool split = false;
  for (int sgi = m->nckpt - 1; sgi >= 0 && e == hipSuccess; --sgi) {
    const int m0 = sgi * K;
    const int cnt = int(std::min<long long>(K, steps - m0));
    // recompute the segment's pre-collision fields from its checkpoint, in
    // place: step i injects into slot i, collides it, and sweeps into slot i + 1
    e = hipMemcpyAsync(seg, m->ckpt + NV * sgi, NV * 4, hipMemcpyDeviceToDevice, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e == hipSuccess) e = hipMemcpy(m->step_ctr, &m0, 4, hipMemcpyHostToDevice);
    for (int i = 0; i < cnt && e == hipSuccess; ++i) {
      float* xi = seg + NV * i;
      float* xn = i + 1 < cnt ? seg + NV * (i + 1) : m->X;
      if (m->npairs > 0) {
        InjectArgs ia{xi, f.Vp, m->src_pairs, m->npairs, m->qdev, m->cap, m->step_ctr, m->budget};
        e = launch_inject(ia, m->stream);
      }
      CollideArgs ca{xi, m->Y, m->P, m->Prow, m->Phi, m->Plo, m->a, m->b, f.Vp, f.NP, m->cpart};
      if (e == hipSuccess) e = launch_collide(ca, f, 0, 0, m->stream);
      SweepArgs sa{m->Y, xn, f.Vp, f.V, f.nx, f.ny, f.nz, m->ddirs, m->delta, m->dstride,
                   m->r, m->iface, m->nvox, m->islot, m->icptF, f.ndir, m->step_ctr, m->spart};
      if (e == hipSuccess) e = launch_sweep(sa, f, split, 0, m->sweep_bpd, m->stream);
      ReduceArgs ra{m->cpart, m->cnwg, m->spart, m->snwg, m->Y, f.Vp, m->det_pairs, m->det_first,
                    m->det_vox_dev, m->ndet, m->ddirs, m->r, 0, m->step_ctr, m->budget,
                    m->det_steps, m->cap, m->flag, m->rscratch, m->rdone};
      if (e == hipSuccess) e = launch_reduce(ra, m->stream);
    }
    // adjoint steps backwards through the segment
    for (int i = cnt - 1; i >= 0 && e == hipSuccess; --i) {
      A.xs = seg + NV * i;
      e = launch_adjoint_step(A, m0 + i, m->stream);
    }
  }
  if (e == hipSuccess) e = hipMemcpyAsync(state_field(m), keep, NV * 4, hipMemcpyDeviceToDevice, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e == hipSuccess) {
    const int sd_steps = int(steps);
    e = hipMemcpy(m->step_ctr, &sd_steps, 4, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemcpy(hga.data(), ga, f.V * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(hgb.data(), gb, f.V * 8, hipMemcpyDeviceToHost);
  cleanup();
  if (e != hipSuccess) return device_fail(m, e, "adjoint");
  return TR_OK;
}

// With the moves in the collision kernels (media whose forward step does the
// moves in the collision's epilogue): the recompute runs the forward step's
// kernel on the segment's slots (slot i to slot i + 1, its injection added in
// place in slot i, no detector keeps and no tallies), and each backward step is
// one kernel, the transposed collision of step m with the transposed moves of
// step m - 1 in its epilogue, plus the seeds of step m - 1.
tr_status backward_fused(tr_medium* m, const std::vector<double>& seed, std::vector<double>& hga,
                         std::vector<double>& hgb) {
  const Field& f = m->f;
  const size_t NV = size_t(f.NP) * f.Vp;
  const long long steps = m->steps_done;
  const int K = m->ckpt_every;
  // the tables of the inverse moves
  std::vector<int8_t> dl(size_t(f.ndir) * 2 * m->dstride, 0);
  for (int d = 0; d < f.ndir; ++d)
    for (int q = 0; q < 2; ++q)
      for (int k = 1; k <= m->lat.maxext; ++k)
        dl[(size_t(d) * 2 + q) * m->dstride + k] =
            int8_t(m->lat.off(d, q, k) - m->lat.off(d, q, k - 1));
  std::vector<int> rtab, rdir;
  if (!build_move_tables(m->lat, dl, m->dstride, f.NP, rtab, rdir, true))
    return fail(TR_EINVAL, "no reversed move tables for this lattice");
  hipError_t e = prepare_adjoint_move(f.NP);
  if (e != hipSuccess) return device_fail(m, e, "adjoint set-up");
  float* mu2 = m->alloc<float>(2 * NV);                   // mu_m in half m & 1
  float* seg = m->alloc<float>(NV * (size_t(K) + 1));      // recomputed fields, and one spare
  double* ga = m->alloc<double>(f.Vp);
  double* gb = m->alloc<double>(f.Vp);
  double* sd = m->alloc<double>(std::max<size_t>(seed.size(), 1));
  int* rt = m->alloc<int>(rtab.size());
  unsigned* nodet = m->alloc<unsigned>(size_t(f.Vp / 32));
  auto cleanup = [&]() {
    for (void* p : {(void*)mu2, (void*)seg, (void*)ga, (void*)gb, (void*)sd, (void*)rt,
                    (void*)nodet})
      m->release(p);
  };
  if (!mu2 || !seg || !ga || !gb || !sd || !rt || !nodet) {
    cleanup();
    return fail(TR_ENOMEM, "no device memory for the adjoint");
  }
  e = hipMemsetAsync(mu2, 0, 2 * NV * 4, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(seg, 0, NV * 4 * (size_t(K) + 1), m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(ga, 0, f.Vp * 8, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(gb, 0, f.Vp * 8, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(nodet, 0, size_t(f.Vp / 32) * 4, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e == hipSuccess && !seed.empty())
    e = hipMemcpy(sd, seed.data(), seed.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(rt, rtab.data(), rtab.size() * 4, hipMemcpyHostToDevice);
  std::vector<int> first(m->ndet + 1);
  if (e == hipSuccess)
    e = hipMemcpy(first.data(), m->det_first, first.size() * 4, hipMemcpyDeviceToHost);
  AdjArgs A{nullptr, nullptr, nullptr, nullptr, m->P, m->a, m->b, ga, gb, f.Vp, f.V, f.nx,
            f.ny, f.nz, f.ndir, f.NP, m->ddirs, m->delta, m->dstride, m->det_pairs, 0,
            m->det_vox_dev, sd, int(steps)};
  A.ndet_pairs = first[m->ndet];
  // the forward step's kernel on the slots
  CollideArgs fw{};
  fw.Prow = m->Prow;
  fw.a = m->a;
  fw.b = m->b;
  fw.Vp = f.Vp;
  fw.NP = f.NP;
  fw.part = m->cpart;
  fw.step_ctr = m->step_ctr;
  fw.mvtab = m->mvtab;
  fw.mvdir = m->mvdir;
  fw.dirs = m->ddirs;
  fw.ndir = f.ndir;
  fw.nx = f.nx;
  fw.ny = f.ny;
  fw.nz = f.nz;
  fw.nvox = f.V;
  fw.mvext = m->mvext;
  fw.mvscramble = m->mvscramble;
  fw.mvunscramble = m->mvunscramble;
  fw.mvdet = nodet;
  fw.spart = m->spart;
  fw.mvfixed = 1;
  InjectArgs ia{m->X, f.Vp, m->src_pairs, m->npairs, m->qdev, m->cap, m->step_ctr, m->budget,
                m->ddirs, false, nullptr};
  // the adjoint's moves: reversed tables over the pair of mu halves
  CollideArgs bw = fw;
  bw.pp = mu2;
  bw.mvtab = rt;
  bw.mvfixed = 0;
  // mu_{steps-1}: the seeds of the last step
  if (e == hipSuccess) {
    AdjArgs a0 = A;
    a0.mu = mu2 + size_t((steps - 1) & 1) * NV;
    e = launch_adjoint_seeds(a0, int(steps - 1), m->stream);
  }
  for (int sgi = m->nckpt - 1; sgi >= 0 && e == hipSuccess; --sgi) {
    const int m0 = sgi * K;
    const int cnt = int(std::min<long long>(K, steps - m0));
    e = hipMemcpyAsync(seg, m->ckpt + NV * sgi, NV * 4, hipMemcpyDeviceToDevice, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e == hipSuccess) e = hipMemcpy(m->step_ctr, &m0, 4, hipMemcpyHostToDevice);
    for (int i = 0; i < cnt && e == hipSuccess; ++i) {
      fw.pp = seg + NV * i;
      e = launch_collide_move(fw, ia, f, 0, m->stream);
      if (e == hipSuccess) e = launch_advance_step(m->step_ctr, m->stream);
    }
    for (int i = cnt - 1; i >= 0 && e == hipSuccess; --i) {
      A.xs = seg + NV * i;
      e = launch_adjoint_move_step(A, bw, m0 + i, m->stream);
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e == hipSuccess) {
    const int sd_steps = int(steps);
    e = hipMemcpy(m->step_ctr, &sd_steps, 4, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemcpy(hga.data(), ga, f.V * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(hgb.data(), gb, f.V * 8, hipMemcpyDeviceToHost);
  cleanup();
  if (e != hipSuccess) return device_fail(m, e, "adjoint");
  return TR_OK;
}

}  // namespace

extern "C" {

const char* tr_last_error(void) { return last_error().c_str(); }

size_t tr_bytes_required(const tr_grid_desc* desc, int ndet, int max_steps) {
  std::string err;
  if (!valid_desc(desc, err) || ndet < 0 || max_steps < 0) return 0;
  if (desc->advance == TR_ADVANCE_RETARDED) return 0;   // the history length depends on n
  return base_bytes(desc, ndet, max_steps);
}

size_t tr_bytes_required_n(const tr_grid_desc* desc, const float* n, int ndet, int max_steps) {
  std::string err;
  if (!valid_desc(desc, err) || !n || ndet < 0 || max_steps < 0) return 0;
  const Field f = field_of(desc);
  // the coefficients' set-up resolves the time step and the path ratios; the
  // sizes do not depend on mu_a and mu_s
  std::vector<float> zero(f.V, 0.0f);
  Coefficients co;
  if (!build_coefficients(int(f.V), zero.data(), zero.data(), n, desc->dx_mm, desc->dt_ps,
                          desc->coef, co, err))
    return 0;
  int mode = desc->advance;
  if (mode == TR_ADVANCE_AUTO) mode = co.uniform_n ? TR_ADVANCE_PHASE : TR_ADVANCE_SPLIT;
  if (mode == TR_ADVANCE_PHASE && !co.uniform_n) return 0;
  tr_grid_desc d = *desc;
  d.advance = mode;
  size_t b = base_bytes(&d, ndet, max_steps);
  const std::vector<Vec3> dirs = healpix_ring(desc->nside);
  const Lattice lat = build_lattice(dirs, f.nx, f.ny, f.nz);
  const bool het = (mode == TR_ADVANCE_SPLIT || mode == TR_ADVANCE_RETARDED) && !co.uniform_n;
  if (het) {
    // interception lists and the gather's targets (one per distinct
    // destination of a reflected or refracted share)
    const std::vector<Interception> icpt = interceptions(lat, dirs, n);
    if (!icpt.empty()) {
      std::vector<char> iface(f.V, 0);
      for (const Interception& ic : icpt) iface[ic.v] = 1;
      size_t ni = 0;
      for (char c : iface) ni += c;
      std::map<std::pair<int, long long>, int> tg;
      size_t nsrc = 0;
      for (const Interception& ic : icpt) {
        tg[{ic.d_refl, ic.v}] = 0;
        ++nsrc;
        if (ic.d_refr >= 0) {
          tg[{ic.d_refr, ic.w}] = 0;
          ++nsrc;
        }
      }
      b += size_t(f.Vp) * (1 + 4 + 4);                          // iface, nvox, islot
      b += ni * f.ndir * sizeof(float);                          // icptF
      if (mode == TR_ADVANCE_RETARDED) b += ni * f.ndir * sizeof(float);   // icptW
      b += (3 * tg.size() + 1 + 2 * nsrc) * 4;                   // targets, ptr, sources, weights
    }
  }
  if (mode == TR_ADVANCE_SPLIT || (mode == TR_ADVANCE_RETARDED && het)) {
    // index classes (at most 127 distinct n): class bytes, path ratios, row bitmap
    std::map<float, int> cls;
    for (long long v = 0; v < f.V && cls.size() <= 127; ++v) cls.emplace(n[v], 0);
    if (cls.size() <= 127)
      b += size_t(f.Vp) + 128 * 4 + (size_t(std::min(f.ny * f.nz, kMaxRowBits)) + 31) / 32 * 4;
  }
  if (mode == TR_ADVANCE_RETARDED) {
    // history length: the longest hop in steps, D = dx / (|Omega_a| l_ref) / r_v
    double rmin = 1.0;
    for (double r : co.r) rmin = std::min(rmin, r);
    int maxlag = 0;
    for (int k = 0; k < f.ndir; ++k) {
      const double D = 1.0 / (lat.speed[k] * (co.ell_ref / desc->dx_mm)) / rmin;
      maxlag = std::max(maxlag, int(std::floor(D + 1e-12)));
    }
    b += size_t(maxlag + 1) * f.NP * f.Vp * sizeof(float);     // the ring
    b += 2 * size_t(f.Vp) * sizeof(float) + 3 * size_t(f.NP) * sizeof(float);
    if (het) b += 4 * size_t(f.NP) * 128 * 4;                   // class hop tables
  }
  return b;
}

tr_status tr_create_medium(const tr_grid_desc* desc, const float* mua, const float* mus,
                           const float* n, int arrays_on_device, void* hip_stream,
                           tr_medium** out) {
  if (!out) return fail(TR_EINVAL, "null output pointer");
  *out = nullptr;
  std::string err;
  if (!valid_desc(desc, err)) return fail(TR_EINVAL, err);
  if (!mua || !mus || !n) return fail(TR_EINVAL, "null coefficient array");
  tr_medium* m = new (std::nothrow) tr_medium();
  if (!m) return fail(TR_ENOMEM, "host allocation failed");
  m->desc = *desc;
  m->stream = static_cast<hipStream_t>(hip_stream);
  m->f = field_of(desc);
  const Field& f = m->f;

  std::vector<float> hmua, hmus;
  const float *pa = mua, *ps = mus, *pn = n;
  if (arrays_on_device) {
    hmua.resize(f.V);
    hmus.resize(f.V);
    m->nhost.resize(f.V);
    // on the given stream, after the work the caller queued there (which may
    // be what wrote the arrays)
    hipError_t e = hipMemcpyAsync(hmua.data(), mua, f.V * 4, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hmus.data(), mus, f.V * 4, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(m->nhost.data(), n, f.V * 4, hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
      delete m;
      return fail(TR_EINVAL, std::string("reading device arrays: ") + hipGetErrorString(e));
    }
    pa = hmua.data();
    ps = hmus.data();
  } else {
    m->nhost.assign(n, n + f.V);
  }
  pn = m->nhost.data();

  m->mua_host.assign(pa, pa + f.V);
  m->mus_host.assign(ps, ps + f.V);
  if (!build_coefficients(f.V, pa, ps, pn, desc->dx_mm, desc->dt_ps, desc->coef, m->co, err)) {
    delete m;
    return fail(TR_EINVAL, err);
  }
  m->dt = m->co.dt;
  m->dirs = healpix_ring(desc->nside);
  m->lat = build_lattice(m->dirs, f.nx, f.ny, f.nz);
  int mode = desc->advance;
  if (mode == TR_ADVANCE_AUTO) mode = m->co.uniform_n ? TR_ADVANCE_PHASE : TR_ADVANCE_SPLIT;
  if (mode == TR_ADVANCE_PHASE && !m->co.uniform_n) {
    delete m;
    return fail(TR_EINVAL, "phase advance needs a uniform refractive index");
  }
  if (mode == TR_ADVANCE_RETARDED && !m->co.uniform_n &&
      desc->nside_scatter != 0 && desc->nside_scatter != desc->nside) {
    delete m;
    return fail(TR_EINVAL, "the retarded advance on a two-level angular grid needs a uniform "
                           "refractive index");
  }
  m->rhet = mode == TR_ADVANCE_RETARDED && !m->co.uniform_n;
  m->mode = mode;
  double maxspeed = 0, maxr = 0;
  for (double s : m->lat.speed) maxspeed = std::max(maxspeed, s);
  for (double r : m->co.r) maxr = std::max(maxr, r);
  if (maxspeed * m->co.ell_ref / desc->dx_mm * maxr > 1.0 + 1e-12) {
    delete m;
    return fail(TR_EINVAL, "time step moves light more than one plane per step");
  }
  std::vector<float> P32, PT;
  m->twolevel = desc->nside_scatter != 0 && desc->nside_scatter != desc->nside;
  m->tlfused = m->twolevel && mode == TR_ADVANCE_PHASE;
  int NPm = f.NP;   // rows of the phase matrix the collide kernels use
  if (m->twolevel) {
    m->nc = 12 * desc->nside_scatter * desc->nside_scatter;
    m->NPc = int(round_up(m->nc, 32));
    m->nkids = f.ndir / m->nc;
    NPm = m->NPc;
  }
  const std::vector<Vec3> pdirs = m->twolevel ? healpix_ring(desc->nside_scatter) : m->dirs;
  if (!build_p32(pdirs, desc->g, desc->hg_norm, NPm, P32, PT)) {
    delete m;
    return fail(TR_EINVAL, "phase matrix scaling did not converge");
  }
  if ((mode == TR_ADVANCE_SPLIT || mode == TR_ADVANCE_RETARDED) && !m->co.uniform_n) {
    m->icpt = interceptions(m->lat, m->dirs, pn);
    m->fresnel = !m->icpt.empty();
  }

  // ---- device buffers
  const size_t NV = size_t(f.NP) * f.Vp;
  m->X = m->alloc<float>(2 * NV);
  m->Y = m->X ? m->X + NV : nullptr;
  m->P = m->alloc<float>(size_t(NPm) * NPm);
  m->Prow = m->alloc<float>(size_t(NPm) * NPm);
  m->a = m->alloc<float>(f.Vp);
  m->b = m->alloc<float>(f.Vp);
  m->r = m->alloc<float>(f.Vp);
  m->ddirs = m->alloc<DevDir>(f.ndir);
  m->dstride = m->lat.maxext + 2;
  m->delta = m->alloc<int8_t>(size_t(f.ndir) * 2 * m->dstride);
  m->step_ctr = m->alloc<int>(1);
  m->flag = m->alloc<int>(1);
  m->rscratch = m->alloc<double>(8);
  m->rdone = m->alloc<int>(1);
  m->cnwg = collide_nwg(f, desc->precision);
  m->sweep_bpd = sweep_blocks_per_dir(f, mode == TR_ADVANCE_RETARDED);
  // two-level phase stepping: row blocks in multiples of 8 for the XCD-ordered
  // grid of the fused sweep (each XCD keeps its blocks for every direction)
  if (m->tlfused && f.ny * f.nz >= 8) m->sweep_bpd = std::max(8, m->sweep_bpd / 8 * 8);
  m->snwg = m->sweep_bpd * f.ndir;
  m->cpart = m->alloc<double>(2 * size_t(m->cnwg));
  m->spart = m->alloc<double>(7 * size_t(std::max(m->snwg, m->cnwg)));
  if (desc->precision == 1) {
    m->Phi = m->alloc<uint16_t>(size_t(f.NP) * f.NP);
    m->Plo = m->alloc<uint16_t>(size_t(f.NP) * f.NP);
    m->plocol = m->alloc<float>(f.NP);
  }
  if (!m->X || !m->Y || !m->P || !m->Prow || !m->a || !m->b || !m->r || !m->ddirs || !m->delta ||
      !m->step_ctr || !m->flag || !m->cpart || !m->spart || !m->rscratch || !m->rdone ||
      (desc->precision == 1 && (!m->Phi || !m->Plo || !m->plocol))) {
    delete m;
    return fail(TR_ENOMEM, "device allocation failed");
  }

  std::vector<float> av(f.Vp, 0.0f), bv(f.Vp, 0.0f), rv(f.Vp, 0.0f);
  for (int v = 0; v < f.V; ++v) {
    av[v] = float(m->co.a[v]);
    bv[v] = float(m->co.b[v]);
    rv[v] = float(m->co.r[v]);
  }
  std::vector<DevDir> dd(f.ndir);
  std::vector<int8_t> dl(size_t(f.ndir) * 2 * m->dstride, 0);
  const double nu_scale = m->co.ell_ref / desc->dx_mm;
  for (int d = 0; d < f.ndir; ++d) {
    dd[d].axis = m->lat.axis[d];
    dd[d].sign = m->lat.sign[d];
    dd[d].bax = m->lat.bax[d];
    dd[d].cax = m->lat.cax[d];
    dd[d].nu64 = m->lat.speed[d] * nu_scale;
    dd[d].nu = float(dd[d].nu64);
    dd[d].unitb = 1;
    for (int q = 0; q < 2; ++q)
      for (int k = 1; k <= m->lat.maxext; ++k) {
        const int s = m->lat.off(d, q, k) - m->lat.off(d, q, k - 1);
        dl[(size_t(d) * 2 + q) * m->dstride + k] = int8_t(s);
        if (q == 0 && (s < -1 || s > 1)) dd[d].unitb = 0;
      }
  }
  // retarded advance: a hop takes D_d = dx / (|Omega_a| l_ref) = 1 / nu_d steps
  for (int d = 0; d < f.ndir; ++d) {
    const double D = 1.0 / dd[d].nu64;
    const int lag = int(std::floor(D + 1e-12));
    dd[d].rlag = lag;
    dd[d].rphi = float(std::max(D - lag, 0.0));
    dd[d].rD = float(D);
    dd[d].rinvD = float(1.0 / D);
  }
  m->fast_split = f.nx % 4 == 0;
  for (const DevDir& D : dd) m->fast_split = m->fast_split && D.unitb;
  // this device's allocation-free workspace (tr_step_noalloc), looked up once
  // per device with the device current
  hipError_t e = scratch_address(&m->scratch);
  if (e != hipSuccess) {
    delete m;
    return fail(TR_EDEVICE, std::string("workspace address: ") + hipGetErrorString(e));
  }
  e = prepare_collide(f, desc->precision);
  if (e == hipSuccess) e = hipMemset(m->X, 0, NV * 4);
  if (e == hipSuccess) e = hipMemset(m->Y, 0, NV * 4);
  if (e == hipSuccess) e = hipMemcpy(m->P, PT.data(), PT.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->Prow, P32.data(), P32.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->a, av.data(), av.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->b, bv.data(), bv.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->r, rv.data(), rv.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->ddirs, dd.data(), dd.size() * sizeof(DevDir), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->delta, dl.data(), dl.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->step_ctr, 0, sizeof(int));
  if (e == hipSuccess) e = hipMemset(m->flag, 0, sizeof(int));
  if (e == hipSuccess) e = hipMemset(m->rdone, 0, sizeof(int));
  if (e == hipSuccess && desc->precision == 1) {
    std::vector<uint16_t> hi(P32.size()), lo(P32.size());
    for (size_t i = 0; i < P32.size(); ++i) {
      hi[i] = f32_to_bf16_bits(P32[i]);
      lo[i] = f32_to_bf16_bits(P32[i] - bf16_bits_to_f32(hi[i]));
    }
    if (desc->hg_norm == TR_HG_SINKHORN) conserve_columns_bf16(hi, lo, f.ndir, f.NP);
    // column totals of P_lo (exact in FP64: sums of bf16 values), for the
    // kernels that leave out the P_lo x_lo product and add its column total
    // to the diagonal
    std::vector<float> lc(f.NP, 0.0f);
    for (int k = 0; k < f.NP; ++k) {
      double t = 0.0;
      for (int i = 0; i < f.NP; ++i) t += double(bf16_bits_to_f32(lo[size_t(i) * f.NP + k]));
      lc[k] = float(t);
    }
    e = hipMemcpy(m->Phi, hi.data(), hi.size() * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->Plo, lo.data(), lo.size() * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->plocol, lc.data(), lc.size() * 4, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    delete m;
    return fail(TR_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
  }

  // ---- phase moves in the collision (tables: build_move_tables)
  m->mfused = mode == TR_ADVANCE_PHASE && !m->twolevel && desc->source == TR_SOURCE_EXPLICIT &&
              desc->transport == TR_TRANSPORT_AUTO && use_collide_move(f);
  std::vector<int> tab, dir;
  if (m->mfused) m->mfused = build_move_tables(m->lat, dl, m->dstride, f.NP, tab, dir);
  {
    const int S = m->lat.maxext;
    if (m->mfused) {
      m->mvext = S;
      // tile order multiplier: the first of these primes that does not divide ntiles
      const long long ntiles = f.Vp / 256;
      for (int pr : {257, 263, 269, 271}) {
        if (ntiles % pr != 0) {
          m->mvscramble = pr;
          break;
        }
      }
      // and its inverse modulo ntiles (extended Euclid)
      long long r0 = ntiles, r1 = m->mvscramble % ntiles, t0 = 0, t1 = 1;
      while (r1 != 0) {
        const long long qq = r0 / r1, r2 = r0 - qq * r1, t2 = t0 - qq * t1;
        r0 = r1;
        r1 = r2;
        t0 = t1;
        t1 = t2;
      }
      m->mvunscramble = int(((t0 % ntiles) + ntiles) % ntiles);
      m->mvtab = m->alloc<int>(tab.size());
      m->mvdir = m->alloc<int>(dir.size());
      m->mvdet = m->alloc<unsigned>(size_t(f.Vp / 32));
      if (!m->mvtab || !m->mvdir || !m->mvdet) {
        delete m;
        return fail(TR_ENOMEM, "device allocation failed (move tables)");
      }
      e = hipMemcpy(m->mvtab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(m->mvdir, dir.data(), dir.size() * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemset(m->mvdet, 0, size_t(f.Vp / 32) * 4);
      if (e == hipSuccess) e = prepare_collide_move(f, desc->precision);
      if (e != hipSuccess) {
        delete m;
        return fail(TR_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
      }
    }
  }

  // ---- Fresnel interface tables
  if (m->fresnel) {
    std::vector<uint8_t> iface(f.V, 0);
    std::vector<int> islot(f.V, -1);
    for (const Interception& ic : m->icpt) iface[ic.v] = 1;
    int ni = 0;
    for (int v = 0; v < f.V; ++v)
      if (iface[v]) islot[v] = ni++;
    m->niface = ni;
    // targets: (d_refl, v) gets R F, (d_refr, w) gets (1 - R) F
    std::map<std::pair<int, long long>, std::vector<std::pair<int, float>>> tg;
    // retarded advance: F is the content that reached the interface, a flux of
    // F / D[d][v]; each share becomes content at the hop duration of its new
    // direction and voxel, D[d][v] = D_d n_v / n_ref
    auto hop = [&](int d, long long v) { return (1.0 / dd[d].nu64) / m->co.r[v]; };
    std::vector<float> wsum;
    if (m->rhet) wsum.assign(size_t(ni) * f.ndir, 0.0f);
    for (const Interception& ic : m->icpt) {
      const int slot = islot[ic.v] * f.ndir + ic.d;
      if (m->rhet) {
        const double Dd = hop(ic.d, ic.v);
        const float wr = float(ic.R * hop(ic.d_refl, ic.v) / Dd);
        const float wt = ic.d_refr >= 0 ? float((1.0 - ic.R) * hop(ic.d_refr, ic.w) / Dd) : 0.0f;
        tg[{ic.d_refl, ic.v}].push_back({slot, wr});
        if (ic.d_refr >= 0) tg[{ic.d_refr, ic.w}].push_back({slot, wt});
        wsum[slot] = float(double(wr) + double(wt));
        continue;
      }
      // reflected share R F; refracted share F - R F, encoded as weight -R
      tg[{ic.d_refl, ic.v}].push_back({slot, float(ic.R)});
      if (ic.d_refr >= 0) tg[{ic.d_refr, ic.w}].push_back({slot, -float(ic.R)});
    }
    std::vector<int> td, tv, ptr(1, 0), src;
    std::vector<float> w;
    for (auto& kv : tg) {
      td.push_back(kv.first.first);
      tv.push_back(int(kv.first.second));
      for (auto& sw : kv.second) {
        src.push_back(sw.first);
        w.push_back(sw.second);
      }
      ptr.push_back(int(src.size()));
    }
    m->ntgt = int(td.size());
    m->iface = m->alloc<uint8_t>(f.Vp);
    m->nvox = m->alloc<float>(f.Vp);
    m->islot = m->alloc<int>(f.Vp);
    m->icptF = m->alloc<float>(size_t(ni) * f.ndir);
    m->tgt_d = m->alloc<int>(td.size());
    m->tgt_v = m->alloc<int>(tv.size());
    m->gptr = m->alloc<int>(ptr.size());
    m->gsrc = m->alloc<int>(src.size());
    m->gw = m->alloc<float>(w.size());
    if (!m->iface || !m->nvox || !m->islot || !m->icptF || !m->tgt_d || !m->tgt_v || !m->gptr ||
        !m->gsrc || !m->gw) {
      delete m;
      return fail(TR_ENOMEM, "device allocation failed (interfaces)");
    }
    iface.resize(f.Vp, 0);
    islot.resize(f.Vp, -1);
    std::vector<float> nv(f.Vp, 1.0f);
    std::copy(pn, pn + f.V, nv.begin());
    e = hipMemcpy(m->iface, iface.data(), f.Vp, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->nvox, nv.data(), f.Vp * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->islot, islot.data(), f.Vp * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(m->icptF, 0, size_t(ni) * f.ndir * 4);
    if (e == hipSuccess) e = hipMemcpy(m->tgt_d, td.data(), td.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->tgt_v, tv.data(), tv.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->gptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->gsrc, src.data(), src.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->gw, w.data(), w.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && m->rhet) {
      m->icptW = m->alloc<float>(wsum.size());
      e = m->icptW ? hipMemcpy(m->icptW, wsum.data(), wsum.size() * 4, hipMemcpyHostToDevice)
                   : hipErrorOutOfMemory;
    }
    if (e != hipSuccess) {
      delete m;
      return fail(TR_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
  }
  // ---- two-level angular grid: children lists, coarse buffers
  if (m->twolevel) {
    const std::vector<int> par = healpix_parents(desc->nside, desc->nside_scatter);
    std::vector<int> kids(size_t(m->nc) * m->nkids, -1), fill(m->nc, 0);
    for (int i = 0; i < f.ndir; ++i) {
      const int J = par[i];
      if (J < 0 || J >= m->nc || fill[J] >= m->nkids) {
        delete m;
        return fail(TR_EINVAL, "inconsistent angular hierarchy");
      }
      kids[size_t(J) * m->nkids + fill[J]++] = i;
    }
    Field fc = f;
    fc.ndir = m->nc;
    fc.NP = m->NPc;
    m->cnwg2 = collide_nwg(fc, 0);
    m->M = m->alloc<float>(size_t(m->NPc) * f.Vp);
    m->T = m->alloc<float>(size_t(m->NPc) * f.Vp);
    m->zero = m->alloc<float>(f.Vp);
    m->children = m->alloc<int>(kids.size());
    m->parent = m->alloc<int>(par.size());
    m->cpart2 = m->alloc<double>(2 * size_t(m->cnwg2));
    if (!m->M || !m->T || !m->zero || !m->children || !m->parent || !m->cpart2) {
      delete m;
      return fail(TR_ENOMEM, "device allocation failed (two-level grid)");
    }
    e = hipMemset(m->M, 0, size_t(m->NPc) * f.Vp * 4);
    if (e == hipSuccess) e = hipMemset(m->T, 0, size_t(m->NPc) * f.Vp * 4);
    if (e == hipSuccess) e = hipMemset(m->zero, 0, f.Vp * 4);
    if (e == hipSuccess) e = hipMemcpy(m->children, kids.data(), kids.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->parent, par.data(), par.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = prepare_collide(fc, 0);
    if (e != hipSuccess) {
      delete m;
      return fail(TR_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    // the budget partials come from the coarse sums, one pair per workgroup
    TwoLevelArgs probe{};
    probe.nc = m->nc;
    probe.V = f.V;
    m->release(m->cpart);
    m->cnwg = int(coarse_sum_workgroups(probe));
    m->cpart = m->alloc<double>(2 * size_t(m->cnwg));
    if (!m->cpart) {
      delete m;
      return fail(TR_ENOMEM, "device allocation failed (two-level partials)");
    }
  }
  // ---- retarded advance: history ring of collided fields and hop tables
  if (m->mode == TR_ADVANCE_RETARDED) {
    int maxlag = 0;
    std::vector<float> ic(f.NP, 0.0f), iD(f.NP, 0.0f), hDv(f.NP, 0.0f);
    for (int d = 0; d < f.ndir; ++d) {
      maxlag = std::max(maxlag, dd[d].rlag);
      ic[d] = float(1.0 / m->lat.speed[d]);
      iD[d] = dd[d].rinvD;
      hDv[d] = dd[d].rD;
    }
    // a varying index: per direction and index class, the hop's whole steps,
    // fraction, D and 1/D, D = D_d n / n_ref (the class's path ratio r =
    // n_ref / n, rtab)
    std::vector<int> lc;
    std::vector<float> pc, Dc, iDc;
    if (m->rhet) {
      // the index classes of the split-mode class bytes: distinct n in
      // increasing order (at most 127, checked there)
      std::map<float, int> cls;
      for (int v = 0; v < f.V && cls.size() <= 127; ++v) cls.emplace(pn[v], 0);
      if (cls.size() > 127) {
        delete m;
        return fail(TR_EINVAL, "the retarded advance takes at most 127 distinct refractive "
                               "indices");
      }
      int nc = 0;
      for (auto& kv : cls) kv.second = nc++;
      std::vector<double> rcls(128, 0.0);
      std::vector<char> seen(128, 0);
      for (int v = 0; v < f.V; ++v) {
        const int c = cls[pn[v]];
        rcls[c] = m->co.r[v];
        seen[c] = 1;
      }
      lc.assign(size_t(f.NP) * 128, 0);
      pc.assign(size_t(f.NP) * 128, 0.0f);
      Dc.assign(size_t(f.NP) * 128, 0.0f);
      iDc.assign(size_t(f.NP) * 128, 0.0f);
      for (int d = 0; d < f.ndir; ++d)
        for (int c = 0; c < 128; ++c) {
          if (!seen[c]) continue;
          const double D = (1.0 / dd[d].nu64) / rcls[c];
          const int lag = int(std::floor(D + 1e-12));
          lc[size_t(d) * 128 + c] = lag;
          pc[size_t(d) * 128 + c] = float(std::max(D - lag, 0.0));
          Dc[size_t(d) * 128 + c] = float(D);
          iDc[size_t(d) * 128 + c] = float(1.0 / D);
          maxlag = std::max(maxlag, lag);
        }
    }
    m->H = maxlag + 1;
    std::vector<float> mx(f.Vp, 0.0f), om(f.Vp, 0.0f);
    for (int v = 0; v < f.V; ++v) {
      const double mt = double(m->mua_host[v]) + double(m->mus_host[v]);
      mx[v] = float(mt * desc->dx_mm);
      // below 2^-20 optical depth per voxel the hop kernel takes a = 1, b = 0
      om[v] = mt * desc->dx_mm >= 0x1p-20 ? float(double(m->mus_host[v]) / mt) : 0.0f;
    }
    const size_t nring = size_t(m->H) * f.NP * f.Vp;
    m->ring = m->alloc<float>(nring);
    m->mutdx = m->alloc<float>(f.Vp);
    m->omega = m->alloc<float>(f.Vp);
    m->hinvc = m->alloc<float>(f.NP);
    m->hinvD = m->alloc<float>(f.NP);
    m->hD = m->alloc<float>(f.NP);
    if (m->rhet) {
      m->rlagc = m->alloc<int>(lc.size());
      m->rphic = m->alloc<float>(pc.size());
      m->rDc = m->alloc<float>(Dc.size());
      m->rinvDc = m->alloc<float>(iDc.size());
    }
    if (!m->ring || !m->mutdx || !m->omega || !m->hinvc || !m->hinvD || !m->hD ||
        (m->rhet && (!m->rlagc || !m->rphic || !m->rDc || !m->rinvDc))) {
      delete m;
      return fail(TR_ENOMEM, "device allocation failed (history of the retarded advance)");
    }
    e = hipMemset(m->ring, 0, nring * 4);
    if (e == hipSuccess) e = hipMemcpy(m->mutdx, mx.data(), mx.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->omega, om.data(), om.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->hinvc, ic.data(), ic.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->hinvD, iD.data(), iD.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->hD, hDv.data(), hDv.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && m->rhet) {
      e = hipMemcpy(m->rlagc, lc.data(), lc.size() * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(m->rphic, pc.data(), pc.size() * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(m->rDc, Dc.data(), Dc.size() * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = hipMemcpy(m->rinvDc, iDc.data(), iDc.size() * 4, hipMemcpyHostToDevice);
    }
    // (on a two-level grid the hop collision is apply_hop's, from the coarse source)
    if (e == hipSuccess && !m->twolevel) e = prepare_collide_hop(f);
    if (e != hipSuccess) {
      delete m;
      return fail(TR_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
  }
  // ---- implicit source: eigen-decomposition of P and per-voxel weights
  if (desc->source == TR_SOURCE_IMPLICIT) {
    std::vector<double> P64, V64, lam64;
    phase_matrix(m->dirs, desc->g, TR_HG_SINKHORN, P64);
    const int n = f.ndir;
    symmetric_eigen(P64, n, V64, lam64);
    std::vector<float> Vf(size_t(f.NP) * f.NP, 0.0f), lf(f.NP, 0.0f);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) Vf[size_t(i) * f.NP + k] = float(V64[size_t(i) * n + k]);
    for (int k = 0; k < n; ++k) lf[k] = float(lam64[k]);
    std::vector<float> w0f(f.Vp, 0.0f), w1f(f.Vp, 0.0f), cf(f.Vp, 0.0f);
    for (int v = 0; v < f.V; ++v) {
      const double ell = kC0 * m->dt / double(pn[v]);
      const double mt = double(pa[v]) + double(ps[v]);
      const double om = mt > 0 ? double(ps[v]) / mt : 0.0;
      double f0, f1;
      eq9_weights(mt * ell, f0, f1);
      w0f[v] = float(om * f0);
      w1f[v] = float(om * f1);
      cf[v] = float((m->co.a[v] + om * f0) / (1.0 - om * f1));
    }
    m->V = m->alloc<float>(Vf.size());
    m->lam = m->alloc<float>(f.NP);
    m->w0 = m->alloc<float>(f.Vp);
    m->w1 = m->alloc<float>(f.Vp);
    m->cimp = m->alloc<float>(f.Vp);
    if (!m->V || !m->lam || !m->w0 || !m->w1 || !m->cimp) {
      delete m;
      return fail(TR_ENOMEM, "device allocation failed (implicit source)");
    }
    e = hipMemcpy(m->V, Vf.data(), Vf.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->lam, lf.data(), lf.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->w0, w0f.data(), w0f.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->w1, w1f.data(), w1f.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->cimp, cf.data(), cf.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = prepare_collide_implicit(f);
    if (e != hipSuccess) {
      delete m;
      return fail(TR_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
  }
  // ---- split mode: one byte per voxel naming its index class (at most 127
  // distinct values of n) and whether it starts an interception
  if (m->mode == TR_ADVANCE_SPLIT || m->rhet) {
    std::map<float, int> cls;
    for (int v = 0; v < f.V && cls.size() <= 127; ++v) cls.emplace(pn[v], 0);
    if (m->rhet && cls.size() > 127) {
      delete m;
      return fail(TR_EINVAL, "the retarded advance takes at most 127 distinct refractive indices");
    }
    if (cls.size() <= 127) {
      std::vector<float> rt(128, 0.0f);
      std::vector<uint8_t> mb(f.Vp, 0);
      int c = 0;
      for (auto& kv : cls) kv.second = c++;
      for (int v = 0; v < f.V; ++v) {
        const int k = cls[pn[v]];
        rt[k] = float(m->co.r[v]);
        mb[v] = uint8_t(k);
      }
      for (const Interception& ic : m->icpt) mb[ic.v] |= 0x80;
      // background class and the bitmap of rows made of it alone
      std::vector<long long> count(128, 0);
      for (int v = 0; v < f.V; ++v) ++count[mb[v] & 0x7f];
      m->bgcls = unsigned(std::max_element(count.begin(), count.end()) - count.begin());
      const int nrow = std::min(f.ny * f.nz, kMaxRowBits);
      std::vector<uint32_t> rb((nrow + 31) / 32, 0u);
      for (int row = 0; row < nrow; ++row) {
        const uint8_t* p = mb.data() + size_t(row) * f.nx;
        bool bg = true;
        for (int x = 0; x < f.nx && bg; ++x) bg = p[x] == m->bgcls;
        if (bg) rb[row >> 5] |= 1u << (row & 31);
      }
      m->mat = m->alloc<uint8_t>(f.Vp);
      m->rtab = m->alloc<float>(128);
      m->rowbits = m->alloc<uint32_t>(rb.size());
      if (!m->mat || !m->rtab || !m->rowbits) {
        delete m;
        return fail(TR_ENOMEM, "device allocation failed (index classes)");
      }
      e = hipMemcpy(m->mat, mb.data(), f.Vp, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(m->rtab, rt.data(), 128 * 4, hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = hipMemcpy(m->rowbits, rb.data(), rb.size() * 4, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        delete m;
        return fail(TR_EDEVICE, std::string("upload: ") + hipGetErrorString(e));
      }
    }
  }
  tr_status st = ensure_capacity(m, 1024);
  if (st != TR_OK) {
    delete m;
    return st;
  }
  *out = m;
  return TR_OK;
}

tr_status tr_destroy_medium(tr_medium* m) {
  if (!m) return TR_OK;
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  else (void)hipDeviceSynchronize();
  delete m;
  return TR_OK;
}

tr_status tr_set_source(tr_medium* m, int ix, int iy, int w, double cone_deg, double t0_ps,
                        double fwhm_ps, double total_photons) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  if (w != 1 && w != 2) return fail(TR_EINVAL, "w must be 1 or 2");
  if (ix < 0 || iy < 0 || ix + w > m->f.nx || iy + w > m->f.ny)
    return fail(TR_EINVAL, "source voxels outside the top face");
  if (!(fwhm_ps > 0) || !std::isfinite(t0_ps) || !std::isfinite(total_photons) ||
      !std::isfinite(cone_deg))
    return fail(TR_EINVAL, "bad pulse parameters");
  std::vector<int> dirs = cone_set(m->dirs, Vec3{0, 0, 1}, cone_deg);
  std::vector<int> pairs;
  for (int d : dirs)
    for (int dy = 0; dy < w; ++dy)
      for (int dx = 0; dx < w; ++dx) {
        pairs.push_back(d);
        pairs.push_back((iy + dy) * m->f.nx + ix + dx);
      }
  hipError_t e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return device_fail(m, e, "synchronize");
  int* dp = m->alloc<int>(pairs.size());
  if (!dp) return fail(TR_ENOMEM, "device allocation failed");
  e = hipMemcpy(dp, pairs.data(), pairs.size() * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) return device_fail(m, e, "source upload");
  m->release(m->src_pairs);
  m->src_pairs = dp;
  m->npairs = int(pairs.size() / 2);
  m->have_source = true;
  m->src_ix = ix;
  m->src_iy = iy;
  m->src_w = w;
  m->src_cone = cone_deg;
  m->src_t0 = t0_ps;
  m->src_fwhm = fwhm_ps;
  m->src_total = total_photons;
  std::vector<double> qh(m->cap);
  for (int s = 0; s < m->cap; ++s) qh[s] = pulse_weight(s, m->dt, t0_ps, fwhm_ps, total_photons);
  e = hipMemcpy(m->qdev, qh.data(), qh.size() * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) return device_fail(m, e, "pulse upload");
  m->drop_graph();
  return TR_OK;
}

tr_status tr_set_detectors(tr_medium* m, int ndet, const int* face, const int* i, const int* j,
                           double cone_deg, double bin_ps, int nbins) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  if (ndet < 1 || ndet > kMaxDet) return fail(TR_EINVAL, "ndet must be in 1..64");
  if (!face || !i || !j) return fail(TR_EINVAL, "null detector arrays");
  if (!(bin_ps > 0) || nbins < 1) return fail(TR_EINVAL, "bad bins");
  const int ext[3] = {m->f.nx, m->f.ny, m->f.nz};
  std::vector<int> fv, vv;
  std::vector<std::vector<int>> acc;
  static const Vec3 normals[6] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
  for (int k = 0; k < ndet; ++k) {
    if (face[k] < 0 || face[k] > 5) return fail(TR_EINVAL, "bad detector face");
    const int ax = face[k] / 2, side = face[k] % 2;
    const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
    if (i[k] < 0 || i[k] >= ext[o1] || j[k] < 0 || j[k] >= ext[o2])
      return fail(TR_EINVAL, "detector indices outside the face");
    int p[3];
    p[ax] = side ? ext[ax] - 1 : 0;
    p[o1] = i[k];
    p[o2] = j[k];
    fv.push_back(face[k]);
    vv.push_back((p[2] * ext[1] + p[1]) * ext[0] + p[0]);
    if (cone_deg <= 0) {
      std::vector<int> all(m->f.ndir);
      for (int d = 0; d < m->f.ndir; ++d) all[d] = d;
      acc.push_back(all);
    } else {
      acc.push_back(cone_set(m->dirs, normals[face[k]], cone_deg));
    }
  }
  hipError_t e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return device_fail(m, e, "synchronize");
  // detector storage depends on ndet: rebuild the capacity-dependent buffers
  int* old_pairs = m->det_pairs;
  int* old_first = m->det_first;
  int* old_vox = m->det_vox_dev;
  m->ndet = ndet;
  m->det_face = fv;
  m->det_vox = vv;
  m->det_cone = cone_deg;
  m->bin_ps = bin_ps;
  m->nbins = nbins;
  st = upload_detector_pairs(m, acc);
  if (st != TR_OK) return st;
  m->release(old_pairs);
  m->release(old_first);
  m->release(old_vox);
  m->release(m->det_steps);
  m->det_steps = m->alloc<double>(size_t(ndet) * m->cap);
  if (!m->det_steps) return fail(TR_ENOMEM, "device allocation failed");
  e = hipMemset(m->det_steps, 0, size_t(ndet) * m->cap * 8);
  if (e != hipSuccess) return device_fail(m, e, "detector reset");
  m->drop_graph();
  return TR_OK;
}

tr_status tr_reset(tr_medium* m) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  const Field& f = m->f;
  hipError_t e = hipMemsetAsync(m->X, 0, size_t(f.NP) * f.Vp * 4, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->Y, 0, size_t(f.NP) * f.Vp * 4, m->stream);
  if (e == hipSuccess && m->ring)
    e = hipMemsetAsync(m->ring, 0, size_t(m->H) * f.NP * f.Vp * 4, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->budget, 0, size_t(m->cap) * 9 * 8, m->stream);
  if (e == hipSuccess && m->ndet > 0)
    e = hipMemsetAsync(m->det_steps, 0, size_t(m->ndet) * m->cap * 8, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->step_ctr, 0, 4, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->flag, 0, 4, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->rdone, 0, 4, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return device_fail(m, e, "reset");
  m->steps_done = 0;
  return TR_OK;
}

tr_status tr_step(tr_medium* m, int nsteps) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  if (nsteps < 0) return fail(TR_EINVAL, "nsteps < 0");
  if (m->ndet == 0) return fail(TR_ESTATE, "detectors not set");
  st = ensure_capacity(m, m->steps_done + nsteps);
  if (st != TR_OK) return st;
  const Workspace ws = medium_workspace(m);
  int left = nsteps;
  hipError_t e = hipSuccess;
  // Replay a captured graph of kGraphSteps steps where possible (the kernels
  // take the step index from the device counter, so replays need no new
  // arguments); the null stream cannot be captured.
  if (m->stream && left >= kGraphSteps && !m->profiling) {
    if (!m->graph) {
      hipGraph_t g;
      e = hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal);
      for (int s = 0; s < kGraphSteps && e == hipSuccess; ++s) e = queue_step(m, ws);
      hipError_t e2 = hipStreamEndCapture(m->stream, &g);
      if (e == hipSuccess) e = e2;
      if (e == hipSuccess) {
        e = hipGraphInstantiate(&m->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
      }
      if (e != hipSuccess) return device_fail(m, e, "graph capture");
    }
    while (left >= kGraphSteps) {
      e = hipGraphLaunch(m->graph, m->stream);
      if (e != hipSuccess) return device_fail(m, e, "graph launch");
      left -= kGraphSteps;
    }
  }
  for (; left > 0; --left) {
    e = queue_step(m, ws);
    if (e != hipSuccess) return device_fail(m, e, "kernel launch");
  }
  m->steps_done += nsteps;
  return TR_OK;
}

tr_status tr_step_noalloc(tr_medium* m, int nsteps) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  if (nsteps < 0) return fail(TR_EINVAL, "nsteps < 0");
  if (m->ndet == 0) return fail(TR_ESTATE, "detectors not set");
  if (m->steps_done + nsteps > m->cap)
    return fail(TR_EINVAL, "tr_step_noalloc: " + std::to_string(m->steps_done + nsteps) +
                               " steps exceed the record capacity of " + std::to_string(m->cap) +
                               " (tr_step grows it)");
  Workspace ws;
  long long used = 0;
  if (!scratch_workspace(m, &ws, &used))
    return fail(TR_EINVAL, "tr_step_noalloc: the step needs " + std::to_string(used) +
                               " doubles of workspace, more than the " +
                               std::to_string(kScratchDoubles) + " the library holds per device");
  if (nsteps == 0) return TR_OK;
  // the tally kernel's counter must start at zero; the workspace keeps
  // whatever the previous call on this device left
  hipError_t e = launch_zero_fill(ws.rscratch, 9, m->stream);
  if (e != hipSuccess) return device_fail(m, e, "kernel launch");
  for (int left = nsteps; left > 0; --left) {
    e = queue_step(m, ws);
    if (e != hipSuccess) return device_fail(m, e, "kernel launch");
  }
  m->steps_done += nsteps;
  return TR_OK;
}

tr_status tr_synchronize(tr_medium* m) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  hipError_t e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return device_fail(m, e, "synchronize");
  int flag = 0;
  e = hipMemcpy(&flag, m->flag, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return device_fail(m, e, "flag read");
  if (flag & 2) {
    m->poisoned = true;
    return fail(TR_EDEVICE, "step beyond tally capacity");
  }
  if (flag & 1) {
    m->poisoned = true;
    return fail(TR_ENUMERIC, "non-finite photon budget");
  }
  return TR_OK;
}

tr_status tr_solve(tr_medium* m, int nsteps) {
  tr_status st = tr_step(m, nsteps);
  if (st != TR_OK) return st;
  return tr_synchronize(m);
}

tr_status tr_read_detector_steps(tr_medium* m, double* out, size_t n_out) {
  tr_status st = tr_synchronize(m);
  if (st != TR_OK) return st;
  const size_t need = size_t(m->ndet) * m->steps_done;
  if (need == 0) return TR_OK;
  if (!out || n_out < need) return fail(TR_EINVAL, "output too small");
  for (int k = 0; k < m->ndet; ++k) {
    hipError_t e = hipMemcpy(out + size_t(k) * m->steps_done, m->det_steps + size_t(k) * m->cap,
                             m->steps_done * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_fail(m, e, "detector read");
  }
  return TR_OK;
}

tr_status tr_read_detectors(tr_medium* m, double* out, size_t n_out) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  const size_t need = size_t(m->ndet) * m->nbins;
  if (!out || n_out < need) return fail(TR_EINVAL, "output too small");
  std::vector<double> raw(size_t(m->ndet) * m->steps_done);
  st = tr_read_detector_steps(m, raw.data(), raw.size());
  if (st != TR_OK) return st;
  rebin(raw.data(), m->steps_done, m->steps_done, m->ndet, m->dt, m->bin_ps, m->nbins, out);
  return TR_OK;
}

tr_status tr_read_budget(tr_medium* m, double* out, size_t n_out) {
  tr_status st = tr_synchronize(m);
  if (st != TR_OK) return st;
  const size_t need = size_t(9) * m->steps_done;
  if (need == 0) return TR_OK;
  if (!out || n_out < need) return fail(TR_EINVAL, "output too small");
  hipError_t e = hipMemcpy(out, m->budget, need * 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return device_fail(m, e, "budget read");
  return TR_OK;
}

tr_status tr_read_energy(tr_medium* m, float* out, int on_device) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  if (!out) return fail(TR_EINVAL, "null output");
  float* E = on_device ? out : m->alloc<float>(m->f.V);
  if (!E) return fail(TR_ENOMEM, "device allocation failed");
  hipError_t e = launch_energy(state_field(m), m->f.Vp, m->f.ndir, m->f.V, E, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e == hipSuccess && !on_device) e = hipMemcpy(out, E, m->f.V * 4, hipMemcpyDeviceToHost);
  if (!on_device) m->release(E);
  if (e != hipSuccess) return device_fail(m, e, "energy");
  return TR_OK;
}

tr_status tr_get_state(tr_medium* m, float* out, int on_device) {
  tr_status st = tr_synchronize(m);
  if (st != TR_OK) return st;
  if (!out) return fail(TR_EINVAL, "null output");
  // on the medium's stream, so that work the caller queued there is ordered with the copy
  hipError_t e = hipMemcpy2DAsync(out, m->f.V * 4, state_field(m), m->f.Vp * 4, m->f.V * 4,
                                  m->f.ndir,
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                  m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return device_fail(m, e, "state read");
  return TR_OK;
}

tr_status tr_set_state(tr_medium* m, const float* in, int on_device) {
  tr_status st = tr_synchronize(m);
  if (st != TR_OK) return st;
  if (!in) return fail(TR_EINVAL, "null input");
  if (m->ring)
    return fail(TR_EINVAL, "the retarded advance keeps a history of collided fields; "
                           "its state cannot be set");
  hipError_t e = hipMemcpy2DAsync(state_field(m), m->f.Vp * 4, in, m->f.V * 4, m->f.V * 4,
                                  m->f.ndir,
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                  m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return device_fail(m, e, "state write");
  return TR_OK;
}

tr_status tr_state_bytes(tr_medium* m, size_t* bytes) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  if (!bytes) return fail(TR_EINVAL, "null output");
  *bytes = state_bytes(m, m->steps_done);
  return TR_OK;
}

tr_status tr_save_state(tr_medium* m, void* out, size_t n_out) {
  tr_status st = tr_synchronize(m);
  if (st != TR_OK) return st;
  if (!out) return fail(TR_EINVAL, "null output");
  const Field& f = m->f;
  const long long steps = m->steps_done;
  const size_t need = state_bytes(m, steps);
  if (n_out < need) return fail(TR_EINVAL, "output too small for the saved state");
  SavedState h{};
  std::memcpy(h.magic, kStateMagic, 8);
  h.fingerprint = state_fingerprint(m);
  h.steps = steps;
  h.ndir = f.ndir;
  h.nvox = f.V;
  h.ndet = m->ndet;
  h.history = m->H;
  h.total = (long long)need;
  char* p = static_cast<char*>(out);
  std::memcpy(p, &h, sizeof h);
  p += sizeof h;
  const size_t field = size_t(f.ndir) * f.V * sizeof(float), slot = size_t(f.NP) * f.Vp;
  hipError_t e = hipMemcpy2DAsync(p, f.V * 4, state_field(m), f.Vp * 4, f.V * 4, f.ndir,
                                  hipMemcpyDeviceToHost, m->stream);
  p += field;
  for (int s = 0; s < m->H && e == hipSuccess; ++s, p += field)
    e = hipMemcpy2DAsync(p, f.V * 4, m->ring + slot * s, f.Vp * 4, f.V * 4, f.ndir,
                         hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess && steps > 0)
    e = hipMemcpyAsync(p, m->budget, size_t(steps) * 9 * 8, hipMemcpyDeviceToHost, m->stream);
  p += size_t(steps) * 9 * 8;
  for (int k = 0; k < m->ndet && e == hipSuccess && steps > 0; ++k, p += size_t(steps) * 8)
    e = hipMemcpyAsync(p, m->det_steps + size_t(k) * m->cap, size_t(steps) * 8,
                       hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return device_fail(m, e, "state save");
  return TR_OK;
}

tr_status tr_load_state(tr_medium* m, const void* in, size_t n_in) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  if (!in) return fail(TR_EINVAL, "null input");
  const Field& f = m->f;
  SavedState h;
  if (n_in < sizeof h) return fail(TR_EINVAL, "input shorter than a saved state's header");
  std::memcpy(&h, in, sizeof h);
  if (std::memcmp(h.magic, kStateMagic, 8) != 0) return fail(TR_EINVAL, "not a saved state");
  if (h.ndir != f.ndir || h.nvox != f.V || h.ndet != m->ndet || h.history != m->H ||
      h.steps < 0 || h.steps > (1LL << 30))
    return fail(TR_EINVAL, "saved state of another shape (directions, voxels, detectors or "
                           "history)");
  if (h.total != (long long)state_bytes(m, h.steps) || n_in < size_t(h.total))
    return fail(TR_EINVAL, "saved state truncated or of another size");
  if (h.fingerprint != state_fingerprint(m))
    return fail(TR_EINVAL, "saved from a medium with another description, medium arrays, "
                           "source or detectors");
  if ((st = ensure_capacity(m, h.steps)) != TR_OK) return st;
  if ((st = tr_reset(m)) != TR_OK) return st;
  m->steps_done = h.steps;   // the state field follows the step's parity
  m->nckpt = 0;              // checkpoints of an earlier solve no longer apply
  const char* p = static_cast<const char*>(in) + sizeof h;
  const size_t field = size_t(f.ndir) * f.V * sizeof(float), slot = size_t(f.NP) * f.Vp;
  hipError_t e = hipMemcpy2DAsync(state_field(m), f.Vp * 4, p, f.V * 4, f.V * 4, f.ndir,
                                  hipMemcpyHostToDevice, m->stream);
  p += field;
  for (int s = 0; s < m->H && e == hipSuccess; ++s, p += field)
    e = hipMemcpy2DAsync(m->ring + slot * s, f.Vp * 4, p, f.V * 4, f.V * 4, f.ndir,
                         hipMemcpyHostToDevice, m->stream);
  if (e == hipSuccess && h.steps > 0)
    e = hipMemcpyAsync(m->budget, p, size_t(h.steps) * 9 * 8, hipMemcpyHostToDevice, m->stream);
  p += size_t(h.steps) * 9 * 8;
  for (int k = 0; k < m->ndet && e == hipSuccess && h.steps > 0; ++k, p += size_t(h.steps) * 8)
    e = hipMemcpyAsync(m->det_steps + size_t(k) * m->cap, p, size_t(h.steps) * 8,
                       hipMemcpyHostToDevice, m->stream);
  const int ctr = int(h.steps);
  if (e == hipSuccess) e = hipMemcpyAsync(m->step_ctr, &ctr, sizeof ctr, hipMemcpyHostToDevice,
                                          m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return device_fail(m, e, "state load");
  return TR_OK;
}

tr_status tr_solve_checkpointed(tr_medium* m, int nsteps, int ckpt_every) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  if (m->V || m->twolevel || m->ring)
    return fail(TR_EINVAL, "gradients are for the explicit source on one angular grid, "
                           "stepped at or below the crossing time without history");
  if (nsteps < 1 || ckpt_every < 1) return fail(TR_EINVAL, "nsteps and ckpt_every must be >= 1");
  if ((st = tr_reset(m)) != TR_OK) return st;
  const Field& f = m->f;
  const size_t NV = size_t(f.NP) * f.Vp;
  const int nseg = (nsteps + ckpt_every - 1) / ckpt_every;
  m->release(m->ckpt);
  m->ckpt = m->alloc<float>(NV * nseg);
  m->nckpt = 0;
  m->ckpt_steps = 0;
  if (!m->ckpt) return fail(TR_ENOMEM, "no device memory for the checkpoints");
  for (int seg = 0; seg < nseg; ++seg) {
    hipError_t e =
        hipMemcpyAsync(m->ckpt + NV * seg, state_field(m), NV * 4, hipMemcpyDeviceToDevice, m->stream);
    if (e != hipSuccess) return device_fail(m, e, "checkpoint");
    if ((st = tr_step(m, std::min(ckpt_every, nsteps - seg * ckpt_every))) != TR_OK) return st;
  }
  m->nckpt = nseg;
  m->ckpt_every = ckpt_every;
  m->ckpt_steps = nsteps;
  return tr_synchronize(m);
}

tr_status tr_backward(tr_medium* m, const double* dL_dbins, float* dmua, float* dmus) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  if (!dL_dbins || !dmua || !dmus) return fail(TR_EINVAL, "null argument");
  if (m->nckpt == 0 || m->ckpt_steps != m->steps_done)
    return fail(TR_ESTATE, "no checkpointed solve of the current steps to differentiate");
  if (m->mode != TR_ADVANCE_PHASE || m->desc.precision != TR_PREC_FP32 || m->f.NP > 192 ||
      m->f.Vp * 4 * 5 >= (1LL << 31))
    return fail(TR_EINVAL, "the adjoint supports phase advance, fp32 and up to 192 directions");
  const Field& f = m->f;
  const long long steps = m->steps_done;
  // seeds dL/d det[k][s]: transpose of the rebinning
  std::vector<double> seed(size_t(m->ndet) * steps, 0.0);
  for (long long s = 0; s < steps; ++s) {
    const double t0 = s * m->dt, t1 = (s + 1) * m->dt;
    const long long j0 = std::max(0LL, (long long)std::floor(t0 / m->bin_ps));
    const long long j1 = std::min<long long>(m->nbins, (long long)std::ceil(t1 / m->bin_ps));
    for (long long j = j0; j < j1; ++j) {
      const double lo = std::max(t0, j * m->bin_ps), hi = std::min(t1, (j + 1) * m->bin_ps);
      if (hi <= lo) continue;
      const double wgt = (hi - lo) / m->dt;
      for (int k = 0; k < m->ndet; ++k)
        seed[size_t(k) * steps + s] += dL_dbins[size_t(k) * m->nbins + j] * wgt;
    }
  }
  std::vector<double> hga(f.V), hgb(f.V);
  st = m->mfused ? backward_fused(m, seed, hga, hgb) : backward_sweep(m, seed, hga, hgb);
  if (st != TR_OK) return st;
  // chain rule through a(mu_a, mu_s), b(mu_a, mu_s)
  for (int v = 0; v < f.V; ++v) {
    const double ma = m->mua_host[v], ms = m->mus_host[v], mt = ma + ms;
    const double ell = kC0 * m->dt / double(m->nhost[v]);
    const double a = std::exp(-mt * ell);
    const double da = -ell * a;
    double db_a, db_s;
    if (m->desc.coef == TR_COEF_PAPER) {
      if (mt > 0) {
        const double om = ms / mt, oneminus = -std::expm1(-mt * ell);
        db_a = -(ms / (mt * mt)) * oneminus + om * ell * a;
        db_s = (ma / (mt * mt)) * oneminus + om * ell * a;
      } else {
        db_a = 0.0;
        db_s = ell;
      }
    } else {
      const double ea = std::exp(-ma * ell), es = std::exp(-ms * ell);
      db_a = -ell * ea * (1.0 - es);
      db_s = ell * ea * es;
    }
    dmua[v] = float(hga[v] * da + hgb[v] * db_a);
    dmus[v] = float(hga[v] * da + hgb[v] * db_s);
  }
  return TR_OK;
}

tr_status tr_profile_begin(tr_medium* m, int max_steps) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  if (max_steps < 1) return fail(TR_EINVAL, "max_steps must be >= 1");
  m->free_events();
  const size_t pairs = size_t(max_steps) * TR_K_COUNT;
  m->prof_ev.resize(2 * pairs, nullptr);
  for (size_t i = 0; i < m->prof_ev.size(); ++i) {
    hipError_t e = hipEventCreate(&m->prof_ev[i]);
    if (e != hipSuccess) {
      m->prof_ev.resize(i);
      m->free_events();
      return fail(TR_ENOMEM, "event creation failed");
    }
  }
  m->prof_kind.assign(pairs, -1);
  m->prof_used = 0;
  m->profiling = true;
  return TR_OK;
}

tr_status tr_profile_end(tr_medium* m, double* kernel_ms, int* launches) {
  tr_status st = check_medium(m);
  if (st != TR_OK) return st;
  if (!m->profiling) return fail(TR_ESTATE, "timing was not started");
  if (!kernel_ms || !launches) return fail(TR_EINVAL, "null output");
  m->profiling = false;
  hipError_t e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) return device_fail(m, e, "synchronize");
  for (int k = 0; k < TR_K_COUNT; ++k) {
    kernel_ms[k] = 0;
    launches[k] = 0;
  }
  for (int i = 0; i < m->prof_used; ++i) {
    float ms = 0;
    e = hipEventElapsedTime(&ms, m->prof_ev[2 * i], m->prof_ev[2 * i + 1]);
    if (e != hipSuccess) return device_fail(m, e, "event timing");
    kernel_ms[m->prof_kind[i]] += ms;
    launches[m->prof_kind[i]] += 1;
  }
  m->free_events();
  return TR_OK;
}

tr_status tr_get_info(tr_medium* m, tr_info* out) {
  if (!m || !out) return fail(TR_EINVAL, "null argument");
  out->ndir = m->f.ndir;
  out->nvox = m->f.V;
  out->mode = m->mode;
  out->ninterceptions = int(m->icpt.size());
  out->dt_ps = m->dt;
  out->steps_done = m->steps_done;
  out->device_bytes = m->bytes;
  out->history = m->H;
  out->moves_fused = m->mfused ? 1 : 0;
  return TR_OK;
}

// ---- host set-up tables ----------------------------------------------------

tr_status tr_host_directions(int nside, double* out) {
  if (nside < 1 || nside > 64 || !out) return fail(TR_EINVAL, "bad nside or output");
  std::vector<Vec3> d = healpix_ring(nside);
  for (size_t i = 0; i < d.size(); ++i) {
    out[3 * i] = d[i].x;
    out[3 * i + 1] = d[i].y;
    out[3 * i + 2] = d[i].z;
  }
  return TR_OK;
}

tr_status tr_host_parents(int nside, int nside_c, int* out) {
  if (!out || nside < 1 || nside > 16 || nside_c < 1 || nside_c > nside || nside % nside_c ||
      ((nside / nside_c) & (nside / nside_c - 1)))
    return fail(TR_EINVAL, "bad nside pair");
  const std::vector<int> par = healpix_parents(nside, nside_c);
  std::copy(par.begin(), par.end(), out);
  return TR_OK;
}

tr_status tr_host_phase_matrix(int nside, double g, int hg_norm, double* out) {
  if (nside < 1 || nside > 16 || !out || !(g > -1 && g < 1)) return fail(TR_EINVAL, "bad arguments");
  std::vector<double> P;
  if (!phase_matrix(healpix_ring(nside), g, hg_norm, P)) return fail(TR_EINVAL, "no convergence");
  std::copy(P.begin(), P.end(), out);
  return TR_OK;
}

tr_status tr_host_lattice(int nside, int nx, int ny, int nz, int* axis, int* sign, int* offset) {
  if (nside < 1 || nside > 16 || nx < 1 || ny < 1 || nz < 1 || !axis || !sign || !offset)
    return fail(TR_EINVAL, "bad arguments");
  Lattice L = build_lattice(healpix_ring(nside), nx, ny, nz);
  std::copy(L.axis.begin(), L.axis.end(), axis);
  std::copy(L.sign.begin(), L.sign.end(), sign);
  std::copy(L.offset.begin(), L.offset.end(), offset);
  return TR_OK;
}

tr_status tr_host_move_tables(int nside, int nx, int ny, int nz, int reverse, int* tab, int* dir) {
  if (nside < 1 || nside > 16 || nx < 1 || ny < 1 || nz < 1 || nx > 1023 || ny > 1023 ||
      nz > 1023 || !tab || !dir)
    return fail(TR_EINVAL, "bad arguments");
  const std::vector<Vec3> dirs = healpix_ring(nside);
  const Lattice L = build_lattice(dirs, nx, ny, nz);
  const int ndir = int(dirs.size()), NP = int(round_up(ndir, 32));
  const int dstride = L.maxext + 2;
  std::vector<int8_t> dl(size_t(ndir) * 2 * dstride, 0);
  for (int d = 0; d < ndir; ++d)
    for (int q = 0; q < 2; ++q)
      for (int k = 1; k <= L.maxext; ++k)
        dl[(size_t(d) * 2 + q) * dstride + k] = int8_t(L.off(d, q, k) - L.off(d, q, k - 1));
  std::vector<int> t, dr;
  if (!build_move_tables(L, dl, dstride, NP, t, dr, reverse != 0))
    return fail(TR_EINVAL, "a direction's transverse shifts are not -1, 0, +1 of one sign");
  std::copy(t.begin(), t.end(), tab);
  std::copy(dr.begin(), dr.end(), dir);
  return TR_OK;
}

tr_status tr_host_coefficients(const tr_grid_desc* desc, const float* mua, const float* mus,
                               const float* n, double* a, double* b, double* r, double* dt_ps) {
  std::string err;
  if (!valid_desc(desc, err)) return fail(TR_EINVAL, err);
  if (!mua || !mus || !n || !a || !b || !r || !dt_ps) return fail(TR_EINVAL, "null argument");
  Coefficients c;
  const int V = desc->nx * desc->ny * desc->nz;
  if (!build_coefficients(V, mua, mus, n, desc->dx_mm, desc->dt_ps, desc->coef, c, err))
    return fail(TR_EINVAL, err);
  std::copy(c.a.begin(), c.a.end(), a);
  std::copy(c.b.begin(), c.b.end(), b);
  std::copy(c.r.begin(), c.r.end(), r);
  *dt_ps = c.dt;
  return TR_OK;
}

tr_status tr_host_cone_set(int nside, double ax, double ay, double az, double cone_deg, int* out,
                           int cap, int* count) {
  if (nside < 1 || nside > 16 || !out || !count) return fail(TR_EINVAL, "bad arguments");
  std::vector<int> s = cone_set(healpix_ring(nside), Vec3{ax, ay, az}, cone_deg);
  *count = int(s.size());
  if (int(s.size()) > cap) return fail(TR_EINVAL, "output too small");
  std::copy(s.begin(), s.end(), out);
  return TR_OK;
}

tr_status tr_host_pulse(double dt_ps, double t0_ps, double fwhm_ps, double total, int m0, int count,
                        double* out) {
  if (!(dt_ps > 0) || !(fwhm_ps > 0) || count < 0 || m0 < 0 || !out)
    return fail(TR_EINVAL, "bad arguments");
  for (int i = 0; i < count; ++i) out[i] = pulse_weight(m0 + i, dt_ps, t0_ps, fwhm_ps, total);
  return TR_OK;
}

tr_status tr_host_interceptions(const tr_grid_desc* desc, const float* n, int* d, int* v, int* w,
                                double* R, int* d_refl, int* d_refr, int cap, int* count) {
  std::string err;
  if (!valid_desc(desc, err)) return fail(TR_EINVAL, err);
  if (!n || !count) return fail(TR_EINVAL, "null argument");
  std::vector<Vec3> dirs = healpix_ring(desc->nside);
  Lattice L = build_lattice(dirs, desc->nx, desc->ny, desc->nz);
  std::vector<Interception> ic = interceptions(L, dirs, n);
  *count = int(ic.size());
  if (int(ic.size()) > cap) return TR_OK;
  if (!d || !v || !w || !R || !d_refl || !d_refr) return fail(TR_EINVAL, "null argument");
  for (size_t i = 0; i < ic.size(); ++i) {
    d[i] = ic[i].d;
    v[i] = int(ic[i].v);
    w[i] = int(ic[i].w);
    R[i] = ic[i].R;
    d_refl[i] = ic[i].d_refl;
    d_refr[i] = ic[i].d_refr;
  }
  return TR_OK;
}

}  // extern "C"
