// Continuous-batching server of forward solves (tr_server_* in include/trinity.h).
//
// Requests are queued on submit, admitted in arrival order whenever a slot and
// enough of the device-memory budget are free, and stepped together: every
// server step runs the batched inject / collide / sweep / tally kernels over
// the work lists of all requests on the device.  The work lists live in device
// memory, so the captured graph of server steps stays valid while requests
// join and leave; the host rewrites the lists between graph replays.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "device.hpp"
#include "host_setup.hpp"
#include "trinity.h"

using namespace trinity;

namespace {

using Clock = std::chrono::steady_clock;
constexpr int kSrvGraphSteps = 8;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
  long long id = 0;
  int status = TR_REQ_QUEUED;
  std::string error;
  tr_grid_desc desc{};
  Field f{};
  int nsteps = 0;
  // host tables (built at submit)
  Coefficients co;
  std::vector<DevDir> dirs;
  std::vector<int8_t> delta;
  int dstride = 0;
  std::vector<int> src_pairs;
  std::vector<double> q;
  std::vector<int> det_pairs, det_first, det_vox;
  int ndet = 0;
  double bin_ps = 1.0;
  int nbins = 0;
  size_t bytes = 0;
  int bpd = 0, ntiles = 0;
  // phase moves in the collision kernel (build_move_tables); the separate
  // sweep where they do not apply
  bool mfused = false;
  std::vector<int> mvtab, mvdir;
  int mvext = 0;
  // device state
  int slot = -1;
  long long steps_done = 0;
  std::vector<void*> dev;
  ReqDev rd{};
  // results
  std::vector<double> det_binned, budget;
  Clock::time_point t_submit, t_start, t_done;
};

// Sizes of a request's device buffers, in allocation order.
struct Layout {
  size_t X, Y, a, b, dirs, delta, src, q, dpairs, dfirst, dvox, budget, dsteps, ints, scratch,
      cpart, spart, mvtab, mvdir, mvdet;
  size_t total() const {
    return X + Y + a + b + dirs + delta + src + q + dpairs + dfirst + dvox + budget + dsteps +
           ints + scratch + cpart + spart + mvtab + mvdir + mvdet;
  }
};

Layout layout_of(const Request& r) {
  Layout L;
  const Field& f = r.f;
  L.X = L.Y = size_t(f.NP) * f.Vp * 4;
  if (r.mfused) {   // both fields in one allocation
    L.X *= 2;
    L.Y = 0;
  }
  L.a = L.b = size_t(f.Vp) * 4;
  L.dirs = size_t(f.ndir) * sizeof(DevDir);
  L.delta = r.delta.size();
  L.src = std::max<size_t>(r.src_pairs.size(), 2) * 4;
  L.q = size_t(r.nsteps) * 8;
  L.dpairs = std::max<size_t>(r.det_pairs.size(), 2) * 4;
  L.dfirst = r.det_first.size() * 4;
  L.dvox = std::max<size_t>(r.det_vox.size(), 1) * 4;
  L.budget = size_t(r.nsteps) * 9 * 8;
  L.dsteps = size_t(std::max(r.ndet, 1)) * r.nsteps * 8;
  L.ints = 3 * 4;
  L.scratch = 8 * 8;
  L.cpart = 2 * size_t(r.ntiles) * 8;
  L.spart = 7 * std::max(size_t(f.ndir) * r.bpd, size_t(r.ntiles)) * 8;
  L.mvtab = r.mvtab.size() * 4;
  L.mvdir = r.mvdir.size() * 4;
  L.mvdet = r.mfused ? size_t(f.Vp / 32) * 4 : 0;
  return L;
}

}  // namespace

struct tr_server {
  tr_server_desc desc{};
  hipStream_t stream = nullptr;
  int ndir = 0, NP = 0;
  std::vector<Vec3> dirs;
  float* Prow = nullptr;
  ReqDev* d_reqs = nullptr;
  int* d_citems = nullptr;
  int* d_sitems = nullptr;
  int* d_counts = nullptr;
  size_t cap_c = 0, cap_s = 0;
  std::vector<Request*> slots;
  std::deque<Request*> pending;
  std::map<long long, Request*> all;
  size_t used = 0;
  long long next_id = 1;
  hipGraphExec_t graph = nullptr;
  bool poisoned = false;

  ~tr_server() {
    if (graph) (void)hipGraphExecDestroy(graph);
    for (auto& kv : all) {
      for (void* p : kv.second->dev) (void)hipFree(p);
      delete kv.second;
    }
    (void)hipFree(Prow);
    (void)hipFree(d_reqs);
    (void)hipFree(d_citems);
    (void)hipFree(d_sitems);
    (void)hipFree(d_counts);
  }
};

namespace {

tr_status srv_device_fail(tr_server* s, hipError_t e, const char* what) {
  s->poisoned = true;
  return fail(TR_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Validate a request and build its host tables (FP64 set-up, as for a medium).
tr_status build_request(const tr_server* s, const tr_request* q, Request& r) {
  if (!q) return fail(TR_EINVAL, "null request");
  r.desc = tr_grid_desc{q->nx, q->ny, q->nz, q->dx_mm, s->desc.nside, s->desc.g, q->dt_ps,
                        s->desc.hg_norm, s->desc.coef, TR_ADVANCE_PHASE, TR_PREC_FP32};
  std::string err;
  if (!valid_desc(&r.desc, err)) return fail(TR_EINVAL, err);
  if (!q->mua || !q->mus || !q->n) return fail(TR_EINVAL, "null coefficient array");
  if (q->nsteps < 1 || q->nsteps > (1 << 24)) return fail(TR_EINVAL, "nsteps must be in 1..2^24");
  r.f = field_of(&r.desc);
  r.nsteps = q->nsteps;
  const Field& f = r.f;
  if (f.Vp * 4 * 5 >= (1LL << 31)) return fail(TR_EINVAL, "grid too large for the server");
  if (!build_coefficients(f.V, q->mua, q->mus, q->n, q->dx_mm, q->dt_ps, s->desc.coef, r.co, err))
    return fail(TR_EINVAL, err);
  if (!r.co.uniform_n) return fail(TR_EINVAL, "the server runs media of uniform refractive index");
  Lattice lat = build_lattice(s->dirs, f.nx, f.ny, f.nz);
  const double nu_scale = r.co.ell_ref / q->dx_mm;
  double maxspeed = 0;
  for (double v : lat.speed) maxspeed = std::max(maxspeed, v);
  if (maxspeed * nu_scale > 1.0 + 1e-12)
    return fail(TR_EINVAL, "time step moves light more than one plane per step");
  r.dirs.resize(f.ndir);
  r.dstride = lat.maxext + 2;
  r.delta.assign(size_t(f.ndir) * 2 * r.dstride, 0);
  for (int d = 0; d < f.ndir; ++d) {
    DevDir& D = r.dirs[d];
    D.axis = lat.axis[d];
    D.sign = lat.sign[d];
    D.bax = lat.bax[d];
    D.cax = lat.cax[d];
    D.nu64 = lat.speed[d] * nu_scale;
    D.nu = float(D.nu64);
    D.unitb = 1;
    for (int qq = 0; qq < 2; ++qq)
      for (int k = 1; k <= lat.maxext; ++k) {
        const int s = lat.off(d, qq, k) - lat.off(d, qq, k - 1);
        r.delta[(size_t(d) * 2 + qq) * r.dstride + k] = int8_t(s);
        if (qq == 0 && (s < -1 || s > 1)) D.unitb = 0;
      }
  }
  // source
  if (q->src_w != 1 && q->src_w != 2) return fail(TR_EINVAL, "src_w must be 1 or 2");
  if (q->src_ix < 0 || q->src_iy < 0 || q->src_ix + q->src_w > f.nx || q->src_iy + q->src_w > f.ny)
    return fail(TR_EINVAL, "source voxels outside the top face");
  if (!(q->fwhm_ps > 0) || !std::isfinite(q->t0_ps) || !std::isfinite(q->total_photons))
    return fail(TR_EINVAL, "bad pulse parameters");
  for (int d : cone_set(s->dirs, Vec3{0, 0, 1}, q->src_cone_deg))
    for (int dy = 0; dy < q->src_w; ++dy)
      for (int dx = 0; dx < q->src_w; ++dx) {
        r.src_pairs.push_back(d);
        r.src_pairs.push_back((q->src_iy + dy) * f.nx + q->src_ix + dx);
      }
  r.q.resize(r.nsteps);
  for (int m = 0; m < r.nsteps; ++m)
    r.q[m] = pulse_weight(m, r.co.dt, q->t0_ps, q->fwhm_ps, q->total_photons);
  // detectors
  if (q->ndet < 1 || q->ndet > kMaxDet) return fail(TR_EINVAL, "ndet must be in 1..64");
  if (!q->det_face || !q->det_i || !q->det_j) return fail(TR_EINVAL, "null detector arrays");
  if (!(q->bin_ps > 0) || q->nbins < 1) return fail(TR_EINVAL, "bad bins");
  static const Vec3 normals[6] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};
  const int ext[3] = {f.nx, f.ny, f.nz};
  r.det_first.push_back(0);
  for (int k = 0; k < q->ndet; ++k) {
    const int face = q->det_face[k];
    if (face < 0 || face > 5) return fail(TR_EINVAL, "bad detector face");
    const int ax = face / 2, o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
    if (q->det_i[k] < 0 || q->det_i[k] >= ext[o1] || q->det_j[k] < 0 || q->det_j[k] >= ext[o2])
      return fail(TR_EINVAL, "detector indices outside the face");
    int p[3];
    p[ax] = face % 2 ? ext[ax] - 1 : 0;
    p[o1] = q->det_i[k];
    p[o2] = q->det_j[k];
    const int v = (p[2] * ext[1] + p[1]) * ext[0] + p[0];
    r.det_vox.push_back(v);
    std::vector<int> acc;
    if (q->det_cone_deg <= 0) {
      for (int d = 0; d < f.ndir; ++d) acc.push_back(d);
    } else {
      acc = cone_set(s->dirs, normals[face], q->det_cone_deg);
    }
    for (int d : acc) {
      int fc;
      if (lat.downwind(d, p[0], p[1], p[2], &fc) < 0 && fc == face) {
        r.det_pairs.push_back(k);
        r.det_pairs.push_back(d);
      }
    }
    r.det_first.push_back(int(r.det_pairs.size() / 2));
  }
  r.ndet = q->ndet;
  r.bin_ps = q->bin_ps;
  r.nbins = q->nbins;
  r.ntiles = int(f.Vp / 256);
  r.bpd = sweep_blocks_per_dir(f, 0);   // phase advance
  if (use_collide_move(f)) r.mfused = build_move_tables(lat, r.delta, r.dstride, f.NP, r.mvtab, r.mvdir);
  if (!r.mfused) r.mvtab.clear(), r.mvdir.clear();
  r.mvext = lat.maxext;
  r.bytes = layout_of(r).total();
  return TR_OK;
}

void release(tr_server* s, Request* r) {
  for (void* p : r->dev) (void)hipFree(p);
  r->dev.clear();
  if (r->slot >= 0) {
    s->slots[r->slot] = nullptr;
    r->slot = -1;
  }
  s->used -= r->bytes;
}

// Allocate and fill a request's device buffers and describe them in r.rd.
tr_status admit(tr_server* s, Request* r, int slot) {
  const Layout L = layout_of(*r);
  const size_t sizes[] = {L.X,      L.Y,      L.a,    L.b,     L.dirs,  L.delta, L.src,
                          L.q,      L.dpairs, L.dfirst, L.dvox, L.budget, L.dsteps, L.ints,
                          L.scratch, L.cpart, L.spart,  L.mvtab, L.mvdir,  L.mvdet};
  std::vector<void*> p;
  for (size_t sz : sizes) {
    void* ptr = nullptr;
    if (hipMalloc(&ptr, std::max<size_t>(sz, 8)) != hipSuccess) {
      for (void* q : p) (void)hipFree(q);
      return fail(TR_ENOMEM, "device allocation failed");
    }
    p.push_back(ptr);
  }
  r->dev = p;
  float* X = static_cast<float*>(p[0]);
  float* Y = r->mfused ? X + size_t(r->f.NP) * r->f.Vp : static_cast<float*>(p[1]);
  float* a = static_cast<float*>(p[2]);
  float* b = static_cast<float*>(p[3]);
  DevDir* dd = static_cast<DevDir*>(p[4]);
  int8_t* dl = static_cast<int8_t*>(p[5]);
  int* src = static_cast<int*>(p[6]);
  double* qd = static_cast<double*>(p[7]);
  int* dpairs = static_cast<int*>(p[8]);
  int* dfirst = static_cast<int*>(p[9]);
  int* dvox = static_cast<int*>(p[10]);
  double* budget = static_cast<double*>(p[11]);
  double* dsteps = static_cast<double*>(p[12]);
  int* ints = static_cast<int*>(p[13]);   // step counter, flag, done
  double* scratch = static_cast<double*>(p[14]);
  double* cpart = static_cast<double*>(p[15]);
  double* spart = static_cast<double*>(p[16]);
  int* mvtab = static_cast<int*>(p[17]);
  int* mvdir = static_cast<int*>(p[18]);
  unsigned* mvdet = static_cast<unsigned*>(p[19]);
  const Field& f = r->f;
  std::vector<float> av(f.Vp, 0.0f), bv(f.Vp, 0.0f);
  for (int v = 0; v < f.V; ++v) {
    av[v] = float(r->co.a[v]);
    bv[v] = float(r->co.b[v]);
  }
  hipError_t e = hipMemsetAsync(X, 0, L.X, s->stream);
  if (e == hipSuccess && !r->mfused) e = hipMemsetAsync(Y, 0, L.Y, s->stream);
  if (e == hipSuccess && r->mfused) {
    std::vector<unsigned> bits(size_t(f.Vp / 32), 0u);
    for (int v : r->det_vox) bits[size_t(v) >> 5] |= 1u << (v & 31);
    e = hipMemcpy(mvtab, r->mvtab.data(), L.mvtab, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(mvdir, r->mvdir.data(), L.mvdir, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(mvdet, bits.data(), L.mvdet, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemsetAsync(budget, 0, L.budget, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(dsteps, 0, L.dsteps, s->stream);
  if (e == hipSuccess) e = hipMemsetAsync(ints, 0, L.ints, s->stream);
  if (e == hipSuccess) e = hipMemcpy(a, av.data(), L.a, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b, bv.data(), L.b, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dd, r->dirs.data(), L.dirs, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dl, r->delta.data(), L.delta, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(src, r->src_pairs.data(), r->src_pairs.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(qd, r->q.data(), L.q, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dpairs, r->det_pairs.data(), r->det_pairs.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dfirst, r->det_first.data(), L.dfirst, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dvox, r->det_vox.data(), r->det_vox.size() * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    for (void* q : p) (void)hipFree(q);
    r->dev.clear();
    return srv_device_fail(s, e, "request upload");
  }
  ReqDev& R = r->rd;
  const int npairs = int(r->src_pairs.size() / 2);
  const int snwg = f.ndir * r->bpd;
  R.inj = InjectArgs{X, f.Vp, src, npairs, qd, r->nsteps, ints, budget};
  R.col = CollideArgs{X, Y, nullptr, s->Prow, nullptr, nullptr, a, b, f.Vp, f.NP, cpart};
  R.swp = SweepArgs{Y, X, f.Vp, f.V, f.nx, f.ny, f.nz, dd, dl, r->dstride, nullptr, nullptr,
                    nullptr, nullptr, nullptr, f.ndir, ints, spart};
  R.red = ReduceArgs{cpart, r->ntiles, spart, snwg, Y, f.Vp, dpairs, dfirst, dvox, r->ndet, dd,
                     nullptr, 0, ints, budget, dsteps, r->nsteps, ints + 1, scratch, ints + 2};
  if (r->mfused) {
    // the field alternates between X and Y by step parity; the collision
    // moves, and its per-tile partials hold the transport tallies too
    R.inj.X2 = Y;
    R.col.step_ctr = ints;
    R.col.pp = X;
    R.col.mvtab = mvtab;
    R.col.mvdir = mvdir;
    R.col.dirs = dd;
    R.col.ndir = f.ndir;
    R.col.nx = f.nx;
    R.col.ny = f.ny;
    R.col.nz = f.nz;
    R.col.nvox = f.V;
    R.col.mvext = r->mvext;
    R.col.mvdet = mvdet;
    R.col.spart = spart;
    R.red.snwg = r->ntiles;
    R.red.mvfused = 1;
    R.red.pp0 = X;
    R.red.pp1 = Y;
  }
  R.nsteps = r->nsteps;
  R.ntiles = r->ntiles;
  R.bpd = r->bpd;
  R.live = 1;
  r->slot = slot;
  s->slots[slot] = r;
  s->used += r->bytes;
  r->status = TR_REQ_RUNNING;
  r->t_start = Clock::now();
  return TR_OK;
}

// Read a finished request's records, bin its detectors, free its slot.
tr_status retire(tr_server* s, Request* r) {
  std::vector<double> raw(size_t(r->ndet) * r->nsteps);
  r->budget.resize(size_t(r->nsteps) * 9);
  int flag = 0;
  hipError_t e = hipMemcpy(raw.data(), r->rd.red.det_steps, raw.size() * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(r->budget.data(), r->rd.red.budget, r->budget.size() * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&flag, r->rd.red.flag, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return srv_device_fail(s, e, "request read-out");
  r->det_binned.assign(size_t(r->ndet) * r->nbins, 0.0);
  rebin(raw.data(), r->nsteps, r->nsteps, r->ndet, r->co.dt, r->bin_ps, r->nbins,
        r->det_binned.data());
  if (r->status != TR_REQ_CANCELLED) {
    if (flag) {
      r->status = TR_REQ_FAILED;
      r->error = flag & 1 ? "non-finite photon budget" : "step beyond tally capacity";
    } else {
      r->status = TR_REQ_DONE;
    }
  }
  r->t_done = Clock::now();
  release(s, r);
  return TR_OK;
}

tr_status rebuild_lists(tr_server* s) {
  std::vector<int> citems, sitems;
  for (int slot = 0; slot < int(s->slots.size()); ++slot) {
    Request* r = s->slots[slot];
    if (!r) continue;
    for (int t = 0; t < r->ntiles; ++t) {
      citems.push_back(slot);
      citems.push_back(t);
    }
    if (r->mfused) continue;   // the collision moves the field
    for (int d = 0; d < r->f.ndir; ++d)
      for (int b = 0; b < r->bpd; ++b) {
        sitems.push_back(slot);
        sitems.push_back(d);
        sitems.push_back(b);
        sitems.push_back(0);
      }
  }
  hipError_t e = hipSuccess;
  const size_t nc = citems.size() / 2, ns = sitems.size() / 4;
  if (nc > s->cap_c || ns > s->cap_s) {
    // grow the lists; the graph refers to the old ones
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return srv_device_fail(s, e, "synchronize");
    (void)hipFree(s->d_citems);
    (void)hipFree(s->d_sitems);
    s->d_citems = s->d_sitems = nullptr;
    s->cap_c = std::max(nc, 2 * s->cap_c);
    s->cap_s = std::max(ns, 2 * s->cap_s);
    if (hipMalloc(&s->d_citems, s->cap_c * 8) != hipSuccess ||
        hipMalloc(&s->d_sitems, s->cap_s * 16) != hipSuccess)
      return srv_device_fail(s, hipErrorOutOfMemory, "work list allocation");
    if (s->graph) (void)hipGraphExecDestroy(s->graph);
    s->graph = nullptr;
  }
  std::vector<ReqDev> reqs(s->slots.size());
  for (size_t i = 0; i < s->slots.size(); ++i) {
    if (s->slots[i]) reqs[i] = s->slots[i]->rd;
    else reqs[i].live = 0;
  }
  const int counts[2] = {int(nc), int(ns)};
  // synchronous copies: the lists are rewritten only between step batches
  e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess && nc) e = hipMemcpy(s->d_citems, citems.data(), nc * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess && ns) e = hipMemcpy(s->d_sitems, sitems.data(), ns * 16, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->d_counts, counts, 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->d_reqs, reqs.data(), reqs.size() * sizeof(ReqDev), hipMemcpyHostToDevice);
  if (e != hipSuccess) return srv_device_fail(s, e, "work list upload");
  return TR_OK;
}

hipError_t queue_server_step(tr_server* s) {
  return launch_server_step(s->d_reqs, int(s->slots.size()), s->d_citems, s->d_sitems,
                            s->d_counts, s->Prow, s->NP, s->stream);
}

tr_status check_server(tr_server* s) {
  if (!s) return fail(TR_EINVAL, "null server");
  if (s->poisoned) return fail(TR_ESTATE, "server is poisoned by an earlier device error");
  return TR_OK;
}

}  // namespace

extern "C" {

tr_status tr_server_create(const tr_server_desc* desc, void* hip_stream, tr_server** out) {
  if (!out) return fail(TR_EINVAL, "null output pointer");
  *out = nullptr;
  if (!desc) return fail(TR_EINVAL, "null descriptor");
  if (desc->nside < 1 || desc->nside > 4) return fail(TR_EINVAL, "server nside must be in 1..4");
  if (!(desc->g > -1 && desc->g < 1)) return fail(TR_EINVAL, "g must be in (-1, 1)");
  if (desc->hg_norm != 0 && desc->hg_norm != 1) return fail(TR_EINVAL, "bad hg_norm");
  if (desc->coef != 0 && desc->coef != 1) return fail(TR_EINVAL, "bad coef");
  if (desc->max_slots < 1 || desc->max_slots > 256) return fail(TR_EINVAL, "max_slots must be in 1..256");
  if (desc->budget_bytes == 0) return fail(TR_EINVAL, "budget_bytes must be > 0");
  tr_server* s = new (std::nothrow) tr_server();
  if (!s) return fail(TR_ENOMEM, "host allocation failed");
  s->desc = *desc;
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->ndir = 12 * desc->nside * desc->nside;
  s->NP = int(round_up(s->ndir, 32));
  s->dirs = healpix_ring(desc->nside);
  std::vector<float> P32, PT;
  if (!build_p32(s->dirs, desc->g, desc->hg_norm, s->NP, P32, PT)) {
    delete s;
    return fail(TR_EINVAL, "phase matrix scaling did not converge");
  }
  s->slots.assign(desc->max_slots, nullptr);
  s->cap_c = 4096;
  s->cap_s = 4096;
  hipError_t e = prepare_server(s->NP);
  if (e == hipSuccess) e = hipMalloc(&s->Prow, P32.size() * 4);
  if (e == hipSuccess) e = hipMalloc(&s->d_reqs, size_t(desc->max_slots) * sizeof(ReqDev));
  if (e == hipSuccess) e = hipMalloc(&s->d_citems, s->cap_c * 8);
  if (e == hipSuccess) e = hipMalloc(&s->d_sitems, s->cap_s * 16);
  if (e == hipSuccess) e = hipMalloc(&s->d_counts, 8);
  if (e == hipSuccess) e = hipMemcpy(s->Prow, P32.data(), P32.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(s->d_counts, 0, 8);
  if (e == hipSuccess) e = hipMemset(s->d_reqs, 0, size_t(desc->max_slots) * sizeof(ReqDev));
  if (e != hipSuccess) {
    delete s;
    return fail(TR_ENOMEM, std::string("server set-up: ") + hipGetErrorString(e));
  }
  *out = s;
  return TR_OK;
}

tr_status tr_server_destroy(tr_server* s) {
  if (!s) return TR_OK;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  else (void)hipDeviceSynchronize();
  delete s;
  return TR_OK;
}

tr_status tr_server_request_bytes(const tr_server* s, const tr_request* q, size_t* bytes) {
  if (!s || !bytes) return fail(TR_EINVAL, "null argument");
  Request r;
  tr_status st = build_request(s, q, r);
  if (st != TR_OK) return st;
  *bytes = r.bytes;
  return TR_OK;
}

tr_status tr_server_submit(tr_server* s, const tr_request* q, long long* id) {
  tr_status st = check_server(s);
  if (st != TR_OK) return st;
  if (!id) return fail(TR_EINVAL, "null id");
  Request* r = new (std::nothrow) Request();
  if (!r) return fail(TR_ENOMEM, "host allocation failed");
  st = build_request(s, q, *r);
  if (st != TR_OK) {
    delete r;
    return st;
  }
  if (r->bytes > s->desc.budget_bytes) {
    delete r;
    return fail(TR_ENOMEM, "request needs more device memory than the whole budget");
  }
  r->id = s->next_id++;
  r->t_submit = Clock::now();
  s->all[r->id] = r;
  s->pending.push_back(r);
  *id = r->id;
  return TR_OK;
}

tr_status tr_server_advance(tr_server* s, int max_steps, int* running, int* queued) {
  tr_status st = check_server(s);
  if (st != TR_OK) return st;
  if (max_steps < 0) return fail(TR_EINVAL, "max_steps < 0");
  bool changed = false;
  // retire finished and cancelled requests
  bool any_done = false;
  for (Request* r : s->slots)
    if (r && (r->steps_done >= r->nsteps || r->status == TR_REQ_CANCELLED)) any_done = true;
  if (any_done) {
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return srv_device_fail(s, e, "synchronize");
    for (Request* r : std::vector<Request*>(s->slots))
      if (r && (r->steps_done >= r->nsteps || r->status == TR_REQ_CANCELLED)) {
        if ((st = retire(s, r)) != TR_OK) return st;
        changed = true;
      }
  }
  // admit in arrival order while a slot and the budget allow
  while (!s->pending.empty()) {
    Request* r = s->pending.front();
    if (s->used + r->bytes > s->desc.budget_bytes) break;
    int slot = -1;
    for (int i = 0; i < int(s->slots.size()); ++i)
      if (!s->slots[i]) {
        slot = i;
        break;
      }
    if (slot < 0) break;
    st = admit(s, r, slot);
    if (st == TR_ENOMEM && s->used > 0) break;   // the device is fuller than the budget says
    if (st != TR_OK) return st;
    s->pending.pop_front();
    changed = true;
  }
  if (changed && (st = rebuild_lists(s)) != TR_OK) return st;
  long long left = max_steps;
  int nrun = 0;
  for (Request* r : s->slots)
    if (r && r->status == TR_REQ_RUNNING) {
      left = std::min(left, r->nsteps - r->steps_done);
      ++nrun;
    }
  if (nrun == 0) left = 0;
  const long long nsteps = left;
  hipError_t e = hipSuccess;
  if (s->stream && left >= kSrvGraphSteps) {
    if (!s->graph) {
      hipGraph_t g;
      e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
      for (int k = 0; k < kSrvGraphSteps && e == hipSuccess; ++k) e = queue_server_step(s);
      hipError_t e2 = hipStreamEndCapture(s->stream, &g);
      if (e == hipSuccess) e = e2;
      if (e == hipSuccess) {
        e = hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
      }
      if (e != hipSuccess) return srv_device_fail(s, e, "graph capture");
    }
    while (left >= kSrvGraphSteps) {
      if ((e = hipGraphLaunch(s->graph, s->stream)) != hipSuccess)
        return srv_device_fail(s, e, "graph launch");
      left -= kSrvGraphSteps;
    }
  }
  for (; left > 0; --left)
    if ((e = queue_server_step(s)) != hipSuccess) return srv_device_fail(s, e, "kernel launch");
  for (Request* r : s->slots)
    if (r && r->status == TR_REQ_RUNNING) r->steps_done += nsteps;
  // retire what just finished so its latency does not wait for the next call
  any_done = false;
  for (Request* r : s->slots)
    if (r && r->steps_done >= r->nsteps) any_done = true;
  if (any_done) {
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return srv_device_fail(s, e, "synchronize");
    bool ch = false;
    for (Request* r : std::vector<Request*>(s->slots))
      if (r && r->steps_done >= r->nsteps) {
        if ((st = retire(s, r)) != TR_OK) return st;
        ch = true;
      }
    if (ch && (st = rebuild_lists(s)) != TR_OK) return st;
  }
  int nr = 0;
  for (Request* r : s->slots) nr += r != nullptr;
  if (running) *running = nr;
  if (queued) *queued = int(s->pending.size());
  return TR_OK;
}

tr_status tr_server_info(tr_server* s, long long id, tr_request_info* out) {
  if (!s || !out) return fail(TR_EINVAL, "null argument");
  auto it = s->all.find(id);
  if (it == s->all.end()) return fail(TR_EINVAL, "unknown request id");
  const Request* r = it->second;
  const Clock::time_point now = Clock::now();
  out->status = r->status;
  out->steps_done = r->steps_done;
  out->bytes = r->bytes;
  const bool started = r->status != TR_REQ_QUEUED && r->t_start.time_since_epoch().count() != 0;
  const bool done = r->t_done.time_since_epoch().count() != 0;
  out->queued_ms = ms_between(r->t_submit, started ? r->t_start : (done ? r->t_done : now));
  out->run_ms = started ? ms_between(r->t_start, done ? r->t_done : now) : 0.0;
  return TR_OK;
}

tr_status tr_server_result(tr_server* s, long long id, double* det, size_t n_det, double* budget,
                           size_t n_budget) {
  if (!s) return fail(TR_EINVAL, "null server");
  auto it = s->all.find(id);
  if (it == s->all.end()) return fail(TR_EINVAL, "unknown request id");
  const Request* r = it->second;
  if (r->status == TR_REQ_FAILED) return fail(TR_ENUMERIC, "request failed: " + r->error);
  if (r->status != TR_REQ_DONE) return fail(TR_ESTATE, "request has no result (not done)");
  if (det) {
    if (n_det < r->det_binned.size()) return fail(TR_EINVAL, "detector output too small");
    std::copy(r->det_binned.begin(), r->det_binned.end(), det);
  }
  if (budget) {
    if (n_budget < r->budget.size()) return fail(TR_EINVAL, "budget output too small");
    std::copy(r->budget.begin(), r->budget.end(), budget);
  }
  return TR_OK;
}

tr_status tr_server_cancel(tr_server* s, long long id) {
  tr_status st = check_server(s);
  if (st != TR_OK) return st;
  auto it = s->all.find(id);
  if (it == s->all.end()) return fail(TR_EINVAL, "unknown request id");
  Request* r = it->second;
  if (r->status == TR_REQ_QUEUED) {
    s->pending.erase(std::remove(s->pending.begin(), s->pending.end(), r), s->pending.end());
    r->status = TR_REQ_CANCELLED;
    r->t_done = Clock::now();
  } else if (r->status == TR_REQ_RUNNING) {
    r->status = TR_REQ_CANCELLED;   // freed at the next advance
  }
  return TR_OK;
}

}  // extern "C"
