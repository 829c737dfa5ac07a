// Batched form: one block eigensolver step for many independent systems
// (uneven grids and band counts, real and Bloch) issued as one graph launch.
//
// Independent systems or k-points are the natural unit of parallel work in
// the method (Sec. "Parallelization"). Each system's step is the chain
// project -> Delta H P -> stencil + add-back -> Delta S P -> S~ -> subspace
// matrices -> Cholesky + eigensolve -> rotation; the chains share nothing, so
// they are dealt onto several capture streams (largest first, to the least
// loaded stream) and recorded once into a HIP graph whose branches run
// concurrently. The subspace eigensolves of all systems small enough for the
// one-workgroup solver run between two such phases as one chain of batched
// launches per scalar type (every system in each launch), so their
// latency-bound stages overlap across systems instead of queueing on a few
// hardware queues; larger systems keep their eigensolve in their branch.
// The autotuner times the launch-shape choices of every system and the
// number of branches.
#include <algorithm>
#include <array>
#include <cstring>
#include <initializer_list>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

struct gpaw_batch {
  struct Buf {
    void *P = nullptr, *Hpsi = nullptr, *Spsi = nullptr, *H = nullptr, *S = nullptr,
         *C = nullptr;
  };
  int device = 0;
  std::vector<gpaw_sys *> sys;
  std::vector<Buf> buf;
  int nbranch = 0;  // 0: default
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> joins;
  hipStream_t cap = nullptr;
  hipEvent_t fork = nullptr, fork2 = nullptr;
  std::vector<hipEvent_t> joins2;
  void *jobs[2] = {nullptr, nullptr};  // batched eigensolver job tables (real, complex)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<gpaw_batch_io> key;  // io the graph was recorded with
  int32_t *key_info = nullptr;
  int key_branches = 0;
};

namespace gfd {
namespace {

constexpr int kMaxBranches = 16;
constexpr int kDefaultBranches = 8;

int check_batch(const gpaw_batch *b) {
  if (!b) return fail(GPAW_EINVAL, "batch is NULL");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != b->device)
    return fail(GPAW_EINVAL, "current HIP device differs from the batch's device");
  return GPAW_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
  if (!a || !b) return false;
  const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
  return pa < pb + nb && pb < pa + na;
}

int check_io(const gpaw_batch *b, const gpaw_batch_io *io, const int32_t *info) {
  if (!io) return fail(GPAW_EINVAL, "io must not be NULL");
  if (!info) return fail(GPAW_EINVAL, "info must not be NULL");
  for (size_t i = 0; i < b->sys.size(); ++i) {
    const gpaw_sys *s = b->sys[i];
    const gpaw_batch_io &x = io[i];
    const std::string tag = "system " + std::to_string(i) + ": ";
    if (x.nb < 1 || x.nb > s->max_bands)
      return fail(GPAW_ESHAPE, tag + "nb outside [1, max_bands]");
    if (!x.psi || !x.psi_out || !x.eps)
      return fail(GPAW_EINVAL, tag + "psi, psi_out and eps must not be NULL");
    const size_t es = elem_size(s->dtype);
    const size_t bytes = static_cast<size_t>(x.nb) * s->ng * es;
    const size_t mbytes = static_cast<size_t>(x.nb) * x.nb * mat_elem_size(s->dtype);
    const size_t pbytes = static_cast<size_t>(x.nb) * s->np * es;
    if (overlaps(x.psi_out, bytes, x.psi, bytes))
      return fail(GPAW_EALIAS, tag + "psi_out overlaps psi");
    const void *mats[3] = {x.H_nn, x.S_nn, x.C_nn};
    for (int a = 0; a < 3; ++a)
      for (int c = a + 1; c < 3; ++c)
        if (overlaps(mats[a], mbytes, mats[c], mbytes))
          return fail(GPAW_EALIAS, tag + "H_nn, S_nn and C_nn must not overlap");
    if (overlaps(x.C_nn, mbytes, x.psi_out, bytes))
      return fail(GPAW_EALIAS, tag + "C_nn overlaps psi_out");
    if (x.P_out && s->np > 0 && overlaps(x.P_out, pbytes, x.psi_out, bytes))
      return fail(GPAW_EALIAS, tag + "P_out overlaps psi_out");
  }
  return GPAW_OK;
}

// Whether system i's eigensolve runs in the batched launches.
bool batched_eig(const gpaw_batch *b, size_t i, const gpaw_batch_io &io) {
  return io.nb <= eig_small_max(is_complex(b->sys[i]->dtype));
}

// Part of system i's step on one stream: phase 0 up to the subspace matrices
// (and, for a system outside the batched eigensolve, the rest of the step);
// phase 1 the rotations after the batched eigensolve.
int chain(const gpaw_batch *b, size_t i, const gpaw_batch_io &io, int32_t *info, hipStream_t st,
          int phase) {
  gpaw_sys *s = b->sys[i];
  const gpaw_batch::Buf &w = b->buf[i];
  const int nb = io.nb;
  void *H = io.H_nn ? io.H_nn : w.H;
  void *S = io.S_nn ? io.S_nn : w.S;
  void *C = io.C_nn ? io.C_nn : w.C;
  const void *X = s->np > 0 ? s->ws.X : nullptr;
  const void *XS = s->np > 0 ? s->ws.XS : nullptr;
  int rc;
  const bool batched = batched_eig(b, i, io);
  if (phase == 0) {
    if (s->np > 0) {
      if ((rc = launch_project(s, io.psi, nb, w.P, st)) != GPAW_OK) return rc;
      if ((rc = launch_dmat2(s, w.P, nb, s->ws.X, s->ws.XS, st)) != GPAW_OK) return rc;
    }
    // H~psi and S~psi in one pass
    if ((rc = launch_stencil(s, io.psi, nb, X, w.Hpsi, st, XS, w.Spsi)) != GPAW_OK) return rc;
    if ((rc = launch_subspace(s, io.psi, w.Hpsi, w.Spsi, nb, H, S, st)) != GPAW_OK) return rc;
    if (batched) return GPAW_OK;
    if ((rc = launch_eigh(s, H, S, nb, io.eps, C, info + i, st)) != GPAW_OK) return rc;
  } else if (!batched) {
    return GPAW_OK;
  }
  if ((rc = launch_rotate(s, C, io.psi, nb, s->ng, io.psi_out, st)) != GPAW_OK) return rc;
  if (s->np > 0 && io.P_out)
    if ((rc = launch_rotate(s, C, w.P, nb, s->np, io.P_out, st)) != GPAW_OK) return rc;
  return GPAW_OK;
}

// The whole step of system i on one stream (its eigensolve unbatched).
int full_chain(const gpaw_batch *b, size_t i, const gpaw_batch_io &io, int32_t *info,
               hipStream_t st) {
  int rc;
  if ((rc = chain(b, i, io, info, st, 0)) != GPAW_OK) return rc;
  if (batched_eig(b, i, io)) {
    gpaw_sys *s = b->sys[i];
    const gpaw_batch::Buf &w = b->buf[i];
    if ((rc = launch_eigh(s, io.H_nn ? io.H_nn : w.H, io.S_nn ? io.S_nn : w.S, io.nb, io.eps,
                          io.C_nn ? io.C_nn : w.C, info + i, st)) != GPAW_OK)
      return rc;
  }
  return chain(b, i, io, info, st, 1);
}

// relative cost of one system's step (grid work, contractions, eigensolver latency)
double cost(const gpaw_sys *s, int nb) {
  const double ng = static_cast<double>(s->ng);
  const double c = is_complex(s->dtype) ? 4.0 : 1.0;
  return ng * nb * (40.0 + c * nb) + 4.0e6 + 2.0e3 * nb * nb;
}

void drop_graph(gpaw_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->key.clear();
}

int record(gpaw_batch *b, const gpaw_batch_io *io, int32_t *info, int branches) {
  drop_graph(b);
  const size_t n = b->sys.size();
  branches = std::max(1, std::min<int>(branches, static_cast<int>(std::min<size_t>(n, kMaxBranches))));
  // largest first onto the least loaded branch
  std::vector<size_t> order(n);
  std::iota(order.begin(), order.end(), size_t(0));
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
    return cost(b->sys[x], io[x].nb) > cost(b->sys[y], io[y].nb);
  });
  std::vector<std::vector<size_t>> lanes(branches);
  std::vector<double> load(branches, 0.0);
  for (size_t i : order) {
    const int l = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
    lanes[l].push_back(i);
    load[l] += cost(b->sys[i], io[i].nb);
  }
  // job tables of the batched eigensolves (a synchronous upload, before
  // the capture; a graph recorded earlier may still read the old tables)
  std::vector<EigBatchItem> items[2];
  for (size_t i = 0; i < n; ++i) {
    if (!batched_eig(b, i, io[i])) continue;
    gpaw_sys *s = b->sys[i];
    const gpaw_batch::Buf &w = b->buf[i];
    items[is_complex(s->dtype) ? 1 : 0].push_back(
        EigBatchItem{s, io[i].H_nn ? io[i].H_nn : w.H, io[i].S_nn ? io[i].S_nn : w.S, io[i].nb,
                     io[i].eps, io[i].C_nn ? io[i].C_nn : w.C, info + i});
  }
  GFD_HIP(hipDeviceSynchronize());
  for (int c = 0; c < 2; ++c) {
    if (b->jobs[c]) (void)hipFree(b->jobs[c]);
    b->jobs[c] = nullptr;
    if (items[c].empty()) continue;
    GFD_HIP(hipMalloc(&b->jobs[c], items[c].size() * eig_job_bytes()));
    int rc0 = eigh_batched_prepare(items[c].data(), static_cast<int>(items[c].size()), b->jobs[c]);
    if (rc0 != GPAW_OK) return rc0;
  }
  GFD_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
  int rc = GPAW_OK;
  hipError_t e = hipSuccess;
  // phase 0 on the branches, the batched eigensolves on the capture stream,
  // phase 1 on the branches again; every fork and join is recorded, also
  // after a failed launch, so that no stream is left in capture mode
  for (int phase = 0; phase < 2; ++phase) {
    hipEvent_t fk = phase == 0 ? b->fork : b->fork2;
    e = hipEventRecord(fk, b->cap);
    for (int l = 0; l < branches && e == hipSuccess; ++l) e = hipStreamWaitEvent(b->streams[l], fk, 0);
    if (e != hipSuccess && rc == GPAW_OK) rc = hip_fail(e, "graph fork");
    for (int l = 0; l < branches && rc == GPAW_OK; ++l)
      for (size_t i : lanes[l])
        if ((rc = chain(b, i, io[i], info, b->streams[l], phase)) != GPAW_OK) break;
    std::vector<hipEvent_t> &jn = phase == 0 ? b->joins : b->joins2;
    for (int l = 0; l < branches; ++l) {
      e = hipEventRecord(jn[l], b->streams[l]);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, jn[l], 0);
      if (e != hipSuccess && rc == GPAW_OK) rc = hip_fail(e, "graph join");
    }
    if (phase == 0 && rc == GPAW_OK)
      for (int c = 0; c < 2 && rc == GPAW_OK; ++c)
        rc = launch_eigh_batched(items[c].data(), static_cast<int>(items[c].size()), c == 1,
                                 b->jobs[c], b->cap);
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap, &g);
  if (rc == GPAW_OK && e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
  if (rc == GPAW_OK) {
    e = hipGetLastError();
    if (e != hipSuccess) rc = hip_fail(e, "batched step launch");
  }
  if (rc != GPAW_OK) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return rc;
  }
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    b->exec = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  b->graph = g;
  b->key.assign(io, io + n);
  b->key_info = info;
  b->key_branches = branches;
  return GPAW_OK;
}

bool same_io(const gpaw_batch *b, const gpaw_batch_io *io, const int32_t *info) {
  if (!b->exec || b->key_info != info || b->key.size() != b->sys.size()) return false;
  return std::memcmp(b->key.data(), io, b->key.size() * sizeof(gpaw_batch_io)) == 0;
}

int branches_of(const gpaw_batch *b) {
  return b->nbranch > 0 ? b->nbranch : kDefaultBranches;
}

void free_batch(gpaw_batch *b) {
  drop_graph(b);
  for (auto &w : b->buf) {
    void *p[] = {w.P, w.Hpsi, w.Spsi, w.H, w.S, w.C};
    for (void *q : p)
      if (q) (void)hipFree(q);
  }
  for (hipStream_t st : b->streams) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : b->joins) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : b->joins2) (void)hipEventDestroy(ev);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->fork2) (void)hipEventDestroy(b->fork2);
  for (void *j : b->jobs)
    if (j) (void)hipFree(j);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

// ------------------------------------------------------------------ autotuner
// Mean time of fn over reps launches on stream st after one warm-up launch.
template <typename F>
int time_ms(F fn, hipStream_t st, int reps, float *ms) {
  hipEvent_t a, z;
  GFD_HIP(hipEventCreate(&a));
  GFD_HIP(hipEventCreate(&z));
  int rc = fn();
  if (rc == GPAW_OK) {
    (void)hipEventRecord(a, st);
    for (int r = 0; r < reps && rc == GPAW_OK; ++r) rc = fn();
    (void)hipEventRecord(z, st);
    (void)hipEventSynchronize(z);
    (void)hipEventElapsedTime(ms, a, z);
    *ms /= reps;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(z);
  if (rc == GPAW_OK) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "autotuner launch");
  }
  return rc;
}

// Try each value of one knob, keep the fastest.
template <typename F>
int pick(int *knob, const std::vector<int> &values, F fn, hipStream_t st) {
  int best = *knob;
  float best_ms = 1e30f;
  for (int v : values) {
    *knob = v;
    float ms = 0.0f;
    int rc = time_ms(fn, st, 3, &ms);
    if (rc != GPAW_OK) return rc;
    if (ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  *knob = best;
  return GPAW_OK;
}

int tune_system(gpaw_batch *b, size_t i, const gpaw_batch_io &io, int32_t *info, hipStream_t st) {
  gpaw_sys *s = b->sys[i];
  const gpaw_batch::Buf &w = b->buf[i];
  const int nb = io.nb;
  const bool cplx = is_complex(s->dtype);
  if (s->dtype == GPAW_F32 || s->dtype == GPAW_C64) return GPAW_OK;  // fixed shapes
  s->tune = Tune{};
  int rc;
  // one full chain so P, X, Hpsi, Spsi, C hold valid data for the part timings
  if ((rc = full_chain(b, i, io, info, st)) != GPAW_OK) return rc;
  void *C = io.C_nn ? io.C_nn : w.C;
  const void *X = s->np > 0 ? s->ws.X : nullptr;
  const void *XS = s->np > 0 ? s->ws.XS : nullptr;
  if (s->np > 0)
    if ((rc = pick(&s->tune.prj_nbg, cplx ? std::vector<int>{1, 2} : std::vector<int>{2, 4, 8},
                   [&] { return launch_project(s, io.psi, nb, w.P, st); }, st)) != GPAW_OK)
      return rc;
  if (s->np > 0)
    if ((rc = launch_dmat2(s, w.P, nb, s->ws.X, s->ws.XS, st)) != GPAW_OK) return rc;
  auto stencil = [&] { return launch_stencil(s, io.psi, nb, X, w.Hpsi, st, XS, w.Spsi); };
  {
    // points per lane 1 or 2, each with its cheapest tiles by the cost
    // model, timed together
    std::vector<std::array<int, 3>> shapes;
    for (int ppl : {1, 2}) {
      s->tune.st_ppl = ppl;
      for (const auto &t : stencil_tiles(s, 3)) shapes.push_back({ppl, t.first, t.second});
    }
    std::vector<int> idx;
    for (size_t j = 0; j < shapes.size(); ++j) idx.push_back(static_cast<int>(j));
    int pickj = 0;
    auto by_shape = [&] {
      s->tune.st_ppl = shapes[pickj][0];
      s->tune.st_ty = shapes[pickj][1];
      s->tune.st_tz = shapes[pickj][2];
      return stencil();
    };
    if ((rc = pick(&pickj, idx, by_shape, st)) != GPAW_OK) return rc;
    s->tune.st_ppl = shapes[pickj][0];
    s->tune.st_ty = shapes[pickj][1];
    s->tune.st_tz = shapes[pickj][2];
  }
  std::vector<int> segs = {0};
  for (int v : {1, 2, 4, 8})
    if (v <= std::max(1, s->n[0] / 12)) segs.push_back(v);
  if ((rc = pick(&s->tune.st_nseg, segs, stencil, st)) != GPAW_OK) return rc;
  if ((rc = pick(&s->tune.sub_wgs, {0, 128, 256, 512, 1024},
                 [&] {
                   return launch_subspace(s, io.psi, w.Hpsi, w.Spsi, nb, w.H, w.S, st);
                 },
                 st)) != GPAW_OK)
    return rc;
  if ((rc = pick(&s->tune.rot_rb, cplx ? std::vector<int>{2, 4} : std::vector<int>{4, 8},
                 [&] { return launch_rotate(s, C, io.psi, nb, s->ng, io.psi_out, st); }, st)) !=
      GPAW_OK)
    return rc;
  return GPAW_OK;
}

}  // namespace
}  // namespace gfd

using namespace gfd;

extern "C" {

int gpaw_batch_create(gpaw_sys *const *systems, int32_t nsys, gpaw_batch **out) {
  if (!systems || !out) return fail(GPAW_EINVAL, "systems and out must not be NULL");
  *out = nullptr;
  if (nsys < 1) return fail(GPAW_EINVAL, "nsys must be >= 1");
  int dev = 0;
  GFD_HIP(hipGetDevice(&dev));
  for (int32_t i = 0; i < nsys; ++i) {
    if (!systems[i]) return fail(GPAW_EINVAL, "system " + std::to_string(i) + " is NULL");
    if (systems[i]->device != dev)
      return fail(GPAW_EINVAL, "system " + std::to_string(i) + " lives on another device");
    for (int32_t j = 0; j < i; ++j)
      if (systems[j] == systems[i])
        return fail(GPAW_EINVAL, "a system appears twice in the batch (its workspace would race)");
  }
  gpaw_batch *b = new gpaw_batch();
  b->device = dev;
  b->sys.assign(systems, systems + nsys);
  b->buf.resize(nsys);
  int rc = GPAW_OK;
  for (int32_t i = 0; i < nsys && rc == GPAW_OK; ++i) {
    const gpaw_sys *s = systems[i];
    const size_t es = elem_size(s->dtype);
    const size_t blk = static_cast<size_t>(s->max_bands) * s->ng * es;
    const size_t mat = static_cast<size_t>(s->max_bands) * s->max_bands * mat_elem_size(s->dtype);
    const size_t pb = static_cast<size_t>(s->max_bands) * s->np * es;
    void **dst[] = {&b->buf[i].Hpsi, &b->buf[i].Spsi, &b->buf[i].H, &b->buf[i].S, &b->buf[i].C,
                    &b->buf[i].P};
    const size_t sz[] = {blk, blk, mat, mat, mat, pb};
    for (int k = 0; k < 6 && rc == GPAW_OK; ++k) {
      if (sz[k] == 0) continue;
      hipError_t e = hipMalloc(dst[k], sz[k]);
      if (e != hipSuccess) rc = hip_fail(e, "hipMalloc(batch workspace)");
    }
  }
  hipError_t e = hipSuccess;
  if (rc == GPAW_OK) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (rc == GPAW_OK && e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (rc == GPAW_OK && e == hipSuccess) e = hipEventCreateWithFlags(&b->fork2, hipEventDisableTiming);
  for (int l = 0; l < kMaxBranches && rc == GPAW_OK && e == hipSuccess; ++l) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) b->streams.push_back(st);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->joins.push_back(ev);
    hipEvent_t ev2 = nullptr;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev2, hipEventDisableTiming);
    if (e == hipSuccess) b->joins2.push_back(ev2);
  }
  if (rc == GPAW_OK && e != hipSuccess) rc = hip_fail(e, "batch streams");
  if (rc != GPAW_OK) {
    free_batch(b);
    return rc;
  }
  *out = b;
  return GPAW_OK;
}

void gpaw_batch_destroy(gpaw_batch *b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  free_batch(b);
}

int gpaw_batch_step(gpaw_batch *b, const gpaw_batch_io *io, int32_t *info, void *stream) {
  int rc;
  if ((rc = check_batch(b)) != GPAW_OK) return rc;
  if ((rc = check_io(b, io, info)) != GPAW_OK) return rc;
  if (!same_io(b, io, info)) {
    // the graph reads the caller's buffers by address: re-record when they change
    GFD_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    if ((rc = record(b, io, info, branches_of(b))) != GPAW_OK) return rc;
  }
  GFD_HIP(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
  return GPAW_OK;
}

int gpaw_batch_tune(gpaw_batch *b, const gpaw_batch_io *io, int32_t *info) {
  int rc;
  if ((rc = check_batch(b)) != GPAW_OK) return rc;
  if ((rc = check_io(b, io, info)) != GPAW_OK) return rc;
  drop_graph(b);
  GFD_HIP(hipDeviceSynchronize());
  for (size_t i = 0; i < b->sys.size(); ++i)
    if ((rc = tune_system(b, i, io[i], info, b->cap)) != GPAW_OK) return rc;
  GFD_HIP(hipStreamSynchronize(b->cap));
  // branch count: record and time the whole graph for each candidate
  int best = kDefaultBranches;
  float best_ms = 1e30f;
  const int nmax = static_cast<int>(std::min<size_t>(b->sys.size(), kMaxBranches));
  for (int nbr : {1, 2, 4, 8, 16}) {
    if (nbr > nmax && nbr != 1) continue;
    if ((rc = record(b, io, info, nbr)) != GPAW_OK) return rc;
    float ms = 0.0f;
    rc = time_ms([&] {
      hipError_t e = hipGraphLaunch(b->exec, b->cap);
      return e == hipSuccess ? GPAW_OK : hip_fail(e, "hipGraphLaunch");
    }, b->cap, 3, &ms);
    if (rc != GPAW_OK) return rc;
    if (ms < best_ms) {
      best_ms = ms;
      best = nbr;
    }
  }
  b->nbranch = best;
  if ((rc = record(b, io, info, best)) != GPAW_OK) return rc;
  return GPAW_OK;
}

int gpaw_batch_set_tuning(gpaw_batch *b, const int32_t *in) {
  int rc;
  if ((rc = check_batch(b)) != GPAW_OK) return rc;
  if (!in) return fail(GPAW_EINVAL, "in must not be NULL");
  if (in[0] < 0 || in[0] > kMaxBranches) return fail(GPAW_EINVAL, "graph branches outside [0, 16]");
  // validate everything before changing anything
  for (size_t i = 0; i < b->sys.size(); ++i) {
    const gpaw_sys *s = b->sys[i];
    const int32_t *v = in + 1 + 7 * i;
    const std::string tag = "system " + std::to_string(i) + ": ";
    const bool cplx = is_complex(s->dtype);
    if (s->dtype == GPAW_F32 || s->dtype == GPAW_C64) {
      for (int k = 0; k < 7; ++k)
        if (v[k] != 0) return fail(GPAW_EINVAL, tag + "single-precision systems keep the built-in shapes");
      continue;
    }
    auto one_of = [](int x, std::initializer_list<int> ok) {
      return std::find(ok.begin(), ok.end(), x) != ok.end();
    };
    if (!one_of(v[0], {0, 1, 2})) return fail(GPAW_EINVAL, tag + "stencil points per lane: 0, 1 or 2");
    if (v[1] < 0 || v[2] < 0 || (v[1] == 0) != (v[2] == 0))
      return fail(GPAW_EINVAL, tag + "stencil tile: both sides positive, or both 0");
    if (v[3] < 0 || v[3] > s->n[0]) return fail(GPAW_EINVAL, tag + "stencil x segments outside [0, n0]");
    if (v[4] < 0 || v[4] > 1024) return fail(GPAW_EINVAL, tag + "subspace workgroups outside [0, 1024]");
    if (!(cplx ? one_of(v[5], {0, 2, 4}) : one_of(v[5], {0, 4, 8})))
      return fail(GPAW_EINVAL, tag + "rotation row tiles: complex 2 or 4, real 4 or 8 (or 0)");
    if (!(cplx ? one_of(v[6], {0, 1, 2}) : one_of(v[6], {0, 2, 4, 8})))
      return fail(GPAW_EINVAL, tag + "projection bands: complex 1 or 2, real 2, 4 or 8 (or 0)");
  }
  for (size_t i = 0; i < b->sys.size(); ++i) {
    Tune &t = b->sys[i]->tune;
    const int32_t *v = in + 1 + 7 * i;
    t.st_ppl = v[0];
    t.st_ty = v[1];
    t.st_tz = v[2];
    t.st_nseg = v[3];
    t.sub_wgs = v[4];
    t.rot_rb = v[5];
    t.prj_nbg = v[6];
  }
  b->nbranch = in[0];
  drop_graph(b);  // the next step records with the new shapes
  return GPAW_OK;
}

int gpaw_batch_tuning(const gpaw_batch *b, int32_t *out) {
  if (!b || !out) return fail(GPAW_EINVAL, "batch and out must not be NULL");
  out[0] = branches_of(b);
  for (size_t i = 0; i < b->sys.size(); ++i) {
    const Tune &t = b->sys[i]->tune;
    int32_t *o = out + 1 + 7 * i;
    o[0] = t.st_ppl;
    o[1] = t.st_ty;
    o[2] = t.st_tz;
    o[3] = t.st_nseg;
    o[4] = t.sub_wgs;
    o[5] = t.rot_rb;
    o[6] = t.prj_nbg;
  }
  return GPAW_OK;
}

}  // extern "C"
