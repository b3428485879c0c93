// Serving engine of the C interface: continuous batching of rollout requests
// over the slots (environments) of one batch.
//
// Each request is one environment of the batch for as long as it runs. An
// engine step advances every request in its forward phase by one chunk of
// substeps in one batched forward call (requests at different points of their
// rollouts share the launches; a request that finishes early is frozen for
// the rest of the call), and moves every request in its backward phase one
// chunk back: its chunk's starting state (the internal state, held as F - I,
// and its collider clock) is restored from the checkpoint taken before the
// chunk ran, one recorded forward and one backward run over all such
// requests, and the running cotangent and the FP64 sum of the parameter
// cotangents are carried to the previous chunk. This is the paper's gradient
// checkpointing with recomputation (Section 5.1) at the granularity of a
// request's chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "../../include/mpm.h"
#include "mpm_internal.h"
#include "mpm_kernels.h"

using namespace mpmx;

namespace {

constexpr int64_t kStateBytes = 96;     // x, v, C, F per particle in FP32
constexpr int64_t kGridNodeBytes = 32;  // a slot's grid share per node (mass, momentum, velocity)

struct Req {
  int64_t id = 0;
  mpm_request r{};
  int state = MPM_REQ_QUEUED;
  int err_bits = 0;
  int slot = -1;
  bool bwd = false;           // in the backward phase
  bool finishing = false;     // retire after the step's synchronization
  int remaining = 0;          // forward substeps left
  int nchunks = 0;
  int chunks_run = 0;         // forward chunks taken so far
  int chunk_idx = -1;         // backward: the chunk to undo next
  std::vector<int> chunk_len;
  std::vector<int64_t> chunk_clock;   // the env's collider clock at each chunk's start
  float* ckpt = nullptr;      // nchunks snapshots of snap_floats floats (backward requests)
  int64_t snap_floats = 0;
  float* cot = nullptr;       // running cotangent [N*3 | N*3 | N*9 | N*9] (backward requests)
  double dparams[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double arrival = 0.0, admitted = 0.0, finished = 0.0;
  int64_t nbytes = 0;
  int64_t n() const { return r.env.n_particles; }
};

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

struct mpm_server {
  mpm_server_desc d{};
  bool dry = false;
  mpm_allocator alloc{};
  bool has_alloc = false;
  hipStream_t stream = nullptr;
  mpm_batch* batch = nullptr;
  std::string err;
  std::chrono::steady_clock::time_point t0;
  int64_t next_id = 1;
  std::map<int64_t, Req> reqs;
  std::deque<int64_t> queue;
  std::vector<int64_t> slot_req;   // request id per slot, -1 free
  int64_t used = 0;
  // caller-order cotangents over all slots for the batched backward (in and
  // out), each as four blocks x [R,3], v [R,3], C [R,9], F [R,9], R = capacity rows
  float* cin = nullptr;
  float* cout = nullptr;
  int64_t rows_cap = 0;
  double* dpar = nullptr;          // [n_slots][8] parameter cotangents of one backward
  std::vector<double> dpar_h;
  // statistics
  int64_t submitted = 0, n_done = 0, n_errors = 0, n_cancelled = 0, n_rejected = 0, work = 0, steps = 0;
  int max_running = 0;
  std::vector<double> lat;
  double first_arrival = -1.0, last_finish = 0.0;
};

namespace {

int sfail(mpm_server* s, int code, const std::string& msg) {
  if (s) s->err = msg;
  return code;
}

#define SCHK(s, expr)                                                            \
  do {                                                                           \
    const int _rc = (expr);                                                      \
    if (_rc != MPM_OK) return sfail((s), _rc, std::string(#expr) + ": " + mpm_last_error((s)->batch)); \
  } while (0)

#define SHIP(s, expr)                                                            \
  do {                                                                           \
    hipError_t _e = (expr);                                                      \
    if (_e != hipSuccess) return sfail((s), MPM_DEVICE_ERROR, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

double now_s(const mpm_server* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

void* sal(mpm_server* s, size_t bytes) {
  if (s->dry) return nullptr;
  bytes = (std::max<size_t>(bytes, 256) + 255) & ~size_t(255);
  void* p = nullptr;
  if (s->has_alloc) p = s->alloc.alloc(bytes, s->alloc.ctx);
  else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
  return p;
}

void sfree(mpm_server* s, void* p) {
  if (!p) return;
  if (s->has_alloc) s->alloc.free(p, s->alloc.ctx);
  else (void)hipFree(p);
}

// device bytes a request keeps while admitted: its state and grid share, and
// for a backward its chunk checkpoints (state + caller ids) and running cotangent
int64_t resident_bytes(const mpm_server* s, const mpm_request& r) {
  const int64_t N = r.env.n_particles;
  const int64_t n = r.env.n;
  int64_t b = N * kStateBytes + n * n * n * kGridNodeBytes;
  if (r.backward) b += ceil_div(r.substeps, s->d.chunk) * 25 * 4 * N + N * kStateBytes;
  return b;
}

mpm_env_desc empty_desc(const mpm_server* s) {
  mpm_env_desc e{};
  e.n = s->d.n_cap;
  e.material = MPM_NEOHOOKEAN;
  e.n_particles = 0;
  e.dt = 5e-5f;
  e.gravity[2] = -9.8f;
  e.wall = 3;
  return e;
}

void free_req_buffers(mpm_server* s, Req& q) {
  sfree(s, q.ckpt);
  sfree(s, q.cot);
  q.ckpt = nullptr;
  q.cot = nullptr;
}

// frees the slot and budget of a running request and records its final state
int release(mpm_server* s, Req& q, int state) {
  q.state = state;
  q.finished = now_s(s);
  q.finishing = false;
  if (q.slot >= 0) {
    s->slot_req[q.slot] = -1;
    if (!s->dry) {
      const mpm_env_desc e = empty_desc(s);
      SCHK(s, mpm_configure_env(s->batch, q.slot, &e));
    }
    q.slot = -1;
  }
  s->used -= q.nbytes;
  free_req_buffers(s, q);
  if (state == MPM_REQ_DONE) {
    ++s->n_done;
    s->work += q.n() * (int64_t)q.r.substeps;
    s->lat.push_back(q.finished - q.arrival);
    s->last_finish = std::max(s->last_finish, q.finished);
  } else if (state == MPM_REQ_ERROR) {
    ++s->n_errors;
  } else if (state == MPM_REQ_CANCELLED) {
    ++s->n_cancelled;
  }
  return MPM_OK;
}

int load_slot(mpm_server* s, Req& q) {
  if (s->dry) return MPM_OK;
  mpm_batch* b = s->batch;
  const mpm_request& r = q.r;
  SCHK(s, mpm_configure_env(b, q.slot, &r.env));
  SCHK(s, mpm_set_material(b, q.slot, r.env.material, r.params));
  if (r.has_collider == 2)
    SCHK(s, mpm_set_sphere_collider(b, q.slot, r.c_center, r.c_half[0], r.c_vel, r.c_alpha, r.c_mu));
  else if (r.has_collider == 3)
    SCHK(s, mpm_set_rounded_box_collider(b, q.slot, r.c_center, r.c_half, r.c_round, r.c_vel, r.c_alpha, r.c_mu));
  else if (r.has_collider)
    SCHK(s, mpm_set_box_collider(b, q.slot, r.c_center, r.c_half, r.c_vel, r.c_alpha, r.c_mu));
  for (int k = 0; k < r.n_more; ++k) {
    const mpm_collider& c = r.more[k];
    SCHK(s, mpm_set_collider(b, q.slot, k + 1, c.shape, c.center, c.half, c.radius, c.vel, c.alpha, c.mu_b));
  }
  SCHK(s, mpm_set_particles(b, q.slot, r.x, r.v, r.C, r.F, r.env.n_particles));
  return MPM_OK;
}

int admit(mpm_server* s) {
  while (!s->queue.empty()) {
    auto free_it = std::find(s->slot_req.begin(), s->slot_req.end(), (int64_t)-1);
    if (free_it == s->slot_req.end()) break;
    Req& q = s->reqs.at(s->queue.front());
    if (s->used + q.nbytes > s->d.budget_bytes) break;   // head of line: arrival order is kept
    const int64_t N = q.n();
    if (q.r.backward && !s->dry) {
      q.snap_floats = 25 * N;
      q.ckpt = (float*)sal(s, sizeof(float) * (size_t)(q.nchunks * q.snap_floats));
      q.cot = (float*)sal(s, sizeof(float) * 24 * (size_t)std::max<int64_t>(N, 1));
      if (!q.ckpt || !q.cot) {
        free_req_buffers(s, q);
        break;   // the allocator is out of memory: the request waits
      }
    }
    s->queue.pop_front();
    q.slot = (int)(free_it - s->slot_req.begin());
    *free_it = q.id;
    s->used += q.nbytes;
    q.state = MPM_REQ_RUNNING;
    q.admitted = now_s(s);
    q.remaining = q.r.substeps;
    const int rc = load_slot(s, q);
    if (rc != MPM_OK) {
      q.err_bits = 0;
      release(s, q, MPM_REQ_ERROR);
      return rc;
    }
  }
  int running = 0;
  for (int64_t id : s->slot_req) running += id >= 0;
  s->max_running = std::max(s->max_running, running);
  return MPM_OK;
}

// copies the request's cotangents of the final state into its running cotangent (NULL = 0)
int init_cotangent(mpm_server* s, Req& q) {
  if (s->dry) return MPM_OK;
  const int64_t N = q.n();
  const float* src[4] = {q.r.gx, q.r.gv, q.r.gC, q.r.gF};
  const int64_t width[4] = {3, 3, 9, 9};
  int64_t off = 0;
  for (int k = 0; k < 4; ++k) {
    const size_t bytes = sizeof(float) * (size_t)(width[k] * N);
    if (src[k]) SHIP(s, hipMemcpyAsync(q.cot + off, src[k], bytes, hipMemcpyDeviceToDevice, s->stream));
    else launch_fill_u32(q.cot + off, 0u, width[k] * N, s->stream);
    off += width[k] * N;
  }
  return MPM_OK;
}

int forward_chunk(mpm_server* s) {
  std::vector<int32_t> counts(s->d.n_slots, 0);
  std::vector<int64_t> ids;
  for (int slot = 0; slot < s->d.n_slots; ++slot) {
    const int64_t id = s->slot_req[slot];
    if (id < 0) continue;
    Req& q = s->reqs.at(id);
    if (q.bwd || q.finishing) continue;
    counts[slot] = std::min(s->d.chunk, q.remaining);
    ids.push_back(id);
  }
  if (ids.empty()) return MPM_OK;
  for (int64_t id : ids) {
    Req& q = s->reqs.at(id);
    if (!q.r.backward) continue;
    const int c = q.chunks_run;
    q.chunk_len[c] = counts[q.slot];
    int64_t clock = 0;
    if (!s->dry) SCHK(s, env_snapshot(s->batch, q.slot, q.ckpt + c * q.snap_floats, &clock));
    q.chunk_clock[c] = clock;
  }
  if (!s->dry) SCHK(s, mpm_forward_envs(s->batch, counts.data(), 0));
  for (int64_t id : ids) {
    Req& q = s->reqs.at(id);
    q.remaining -= counts[q.slot];
    ++q.chunks_run;
    if (q.remaining > 0) continue;
    if (!s->dry && (q.r.out_x || q.r.out_v || q.r.out_C || q.r.out_F))
      SCHK(s, mpm_get_particles(s->batch, q.slot, q.r.out_x, q.r.out_v, q.r.out_C, q.r.out_F));
    if (q.r.backward) {
      q.bwd = true;
      q.chunk_idx = q.chunks_run - 1;
      const int rc = init_cotangent(s, q);
      if (rc != MPM_OK) return rc;
    } else {
      q.finishing = true;
    }
  }
  return MPM_OK;
}

// copies rows [row, row + N) of the four caller-order blocks between the
// batch-wide cotangent buffer `all` (capacity R rows) and a request's running
// cotangent `mine` ([N*3 | N*3 | N*9 | N*9])
int copy_rows(mpm_server* s, float* all, float* mine, int64_t row, int64_t N, bool to_all) {
  const int64_t R = s->rows_cap;
  const int64_t width[4] = {3, 3, 9, 9};
  const int64_t block[4] = {0, 3 * R, 6 * R, 15 * R};
  int64_t off = 0;
  for (int k = 0; k < 4; ++k) {
    float* a = all + block[k] + width[k] * row;
    float* m = mine + off;
    const size_t bytes = sizeof(float) * (size_t)(width[k] * N);
    if (bytes) SHIP(s, hipMemcpyAsync(to_all ? a : m, to_all ? m : a, bytes, hipMemcpyDeviceToDevice, s->stream));
    off += width[k] * N;
  }
  return MPM_OK;
}

int backward_chunk(mpm_server* s, std::vector<int64_t>& bwd_ids) {
  std::vector<int32_t> counts(s->d.n_slots, 0);
  for (int slot = 0; slot < s->d.n_slots; ++slot) {
    const int64_t id = s->slot_req[slot];
    if (id < 0) continue;
    Req& q = s->reqs.at(id);
    if (!q.bwd || q.finishing || q.chunk_idx < 0) continue;
    counts[slot] = q.chunk_len[q.chunk_idx];
    bwd_ids.push_back(id);
  }
  if (bwd_ids.empty() || s->dry) return MPM_OK;
  mpm_batch* b = s->batch;
  for (int64_t id : bwd_ids) {
    Req& q = s->reqs.at(id);
    SCHK(s, env_restore(b, q.slot, q.ckpt + q.chunk_idx * q.snap_floats, q.chunk_clock[q.chunk_idx]));
  }
  SCHK(s, mpm_forward_envs(b, counts.data(), MPM_FWD_RECORD));
  const int64_t R = s->rows_cap;
  launch_fill_u32(s->cin, 0u, 24 * R, s->stream);
  for (int64_t id : bwd_ids) {
    Req& q = s->reqs.at(id);
    const int rc = copy_rows(s, s->cin, q.cot, env_row_offset(b, q.slot), q.n(), true);
    if (rc != MPM_OK) return rc;
  }
  SCHK(s, mpm_backward(b, s->cin, s->cin + 3 * R, s->cin + 6 * R, s->cin + 15 * R, s->cout, s->cout + 3 * R,
                       s->cout + 6 * R, s->cout + 15 * R, s->dpar));
  for (int64_t id : bwd_ids) {
    Req& q = s->reqs.at(id);
    const int rc = copy_rows(s, s->cout, q.cot, env_row_offset(b, q.slot), q.n(), false);
    if (rc != MPM_OK) return rc;
  }
  SHIP(s, hipMemcpyAsync(s->dpar_h.data(), s->dpar, sizeof(double) * 8 * s->d.n_slots, hipMemcpyDeviceToHost,
                         s->stream));
  return MPM_OK;
}

// after the step's device work: per-env errors, FP64 parameter-cotangent sums,
// chunk bookkeeping, outputs of finished backwards, retirement
int finish_step(mpm_server* s, const std::vector<int64_t>& bwd_ids) {
  std::vector<int32_t> errs(s->d.n_slots, 0);
  if (!s->dry) {
    const int rc = mpm_sync(s->batch);
    if (rc != MPM_OK && rc != MPM_NONFINITE && rc != MPM_OUT_OF_DOMAIN)
      return sfail(s, rc, std::string("mpm_sync: ") + mpm_last_error(s->batch));
    SCHK(s, mpm_env_errors(s->batch, errs.data()));
  }
  for (int64_t id : bwd_ids) {
    Req& q = s->reqs.at(id);
    for (int k = 0; k < 8; ++k) q.dparams[k] += s->dry ? 0.0 : s->dpar_h[8 * q.slot + k];
    --q.chunk_idx;
    if (q.chunk_idx >= 0) continue;
    if (!s->dry) {
      const int64_t N = q.n();
      float* dst[4] = {q.r.dx0, q.r.dv0, q.r.dC0, q.r.dF0};
      const int64_t width[4] = {3, 3, 9, 9};
      int64_t off = 0;
      for (int k = 0; k < 4; ++k) {
        if (dst[k])
          SHIP(s, hipMemcpyAsync(dst[k], q.cot + off, sizeof(float) * (size_t)(width[k] * N),
                                 hipMemcpyDeviceToDevice, s->stream));
        off += width[k] * N;
      }
    }
    q.finishing = true;
  }
  if (!s->dry) SHIP(s, hipStreamSynchronize(s->stream));
  for (int slot = 0; slot < s->d.n_slots; ++slot) {
    const int64_t id = s->slot_req[slot];
    if (id < 0) continue;
    Req& q = s->reqs.at(id);
    if (errs[slot]) {
      q.err_bits = errs[slot];
      SCHK(s, release(s, q, MPM_REQ_ERROR));
    } else if (q.finishing) {
      SCHK(s, release(s, q, MPM_REQ_DONE));
    }
  }
  return MPM_OK;
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = p / 100.0 * (double)(v.size() - 1);   // linear interpolation between ranks
  const size_t i = (size_t)std::floor(pos);
  const size_t j = std::min(i + 1, v.size() - 1);
  return v[i] + (pos - (double)i) * (v[j] - v[i]);
}

}  // namespace

extern "C" {

int mpm_server_create(const mpm_server_desc* d, const mpm_allocator* a, void* stream, mpm_server** out) {
  if (!d || !out) return MPM_INVALID_ARG;
  *out = nullptr;
  if (d->n_slots < 1 || d->n_cap < 12 || d->n_cap % 4 != 0 || d->n_cap > 1024 || d->n_cap_particles < 1 ||
      d->chunk < 1 || d->budget_bytes < 0 || (d->flags & ~MPM_SERVER_DRY) != 0)
    return MPM_INVALID_ARG;
  if (a && (!a->alloc || !a->free)) return MPM_INVALID_ARG;
  mpm_server* s = new mpm_server();
  s->d = *d;
  s->dry = (d->flags & MPM_SERVER_DRY) != 0;
  if (a) { s->alloc = *a; s->has_alloc = true; }
  s->stream = (hipStream_t)stream;
  s->t0 = std::chrono::steady_clock::now();
  s->slot_req.assign(d->n_slots, -1);
  s->dpar_h.assign(8 * (size_t)d->n_slots, 0.0);
  if (!s->dry) {
    std::vector<mpm_env_desc> envs(d->n_slots, empty_desc(s));
    for (auto& e : envs) e.n_particles = d->n_cap_particles;   // capacities
    mpm_batch_desc bd{};
    bd.n_envs = d->n_slots;
    bd.envs = envs.data();
    bd.max_substeps = d->chunk;
    bd.ckpt_every = d->chunk;
    bd.mode = MPM_MODE_BATCHED;
    int rc = mpm_batch_create(&bd, a, stream, &s->batch);
    if (rc == MPM_OK) {
      const mpm_env_desc e = empty_desc(s);
      for (int i = 0; i < d->n_slots && rc == MPM_OK; ++i) rc = mpm_configure_env(s->batch, i, &e);
    }
    s->rows_cap = (int64_t)d->n_slots * d->n_cap_particles;
    if (rc == MPM_OK) {
      s->cin = (float*)sal(s, sizeof(float) * 24 * (size_t)s->rows_cap);
      s->cout = (float*)sal(s, sizeof(float) * 24 * (size_t)s->rows_cap);
      s->dpar = (double*)sal(s, sizeof(double) * 8 * (size_t)d->n_slots);
      if (!s->cin || !s->cout || !s->dpar) rc = MPM_OUT_OF_MEMORY;
    }
    if (rc == MPM_OK && hipStreamSynchronize(s->stream) != hipSuccess) rc = MPM_DEVICE_ERROR;
    if (rc != MPM_OK) {
      sfree(s, s->cin);
      sfree(s, s->cout);
      sfree(s, s->dpar);
      if (s->batch) mpm_batch_destroy(s->batch);
      delete s;
      return rc;
    }
  }
  *out = s;
  return MPM_OK;
}

int mpm_server_destroy(mpm_server* s) {
  if (!s) return MPM_INVALID_ARG;
  if (!s->dry) (void)hipStreamSynchronize(s->stream);
  for (auto& kv : s->reqs) free_req_buffers(s, kv.second);
  sfree(s, s->cin);
  sfree(s, s->cout);
  sfree(s, s->dpar);
  if (s->batch) mpm_batch_destroy(s->batch);
  delete s;
  return MPM_OK;
}

int mpm_server_submit(mpm_server* s, const mpm_request* r, int64_t* id) {
  if (!s || !r || !id) return MPM_INVALID_ARG;
  const mpm_env_desc& e = r->env;
  if (r->substeps < 1) return sfail(s, MPM_INVALID_ARG, "substeps must be >= 1");
  if (e.n_particles < 0) return sfail(s, MPM_INVALID_ARG, "negative particle count");
  if (e.n_particles > 0 && (!r->x || !r->v || !r->C || !r->F)) return sfail(s, MPM_INVALID_ARG, "null state array");
  if (e.material < 0 || e.material > MPM_FLUID_PAPER) return sfail(s, MPM_INVALID_ARG, "unknown material");
  if (!(r->params[1] > -1.0 && r->params[1] < 0.5)) return sfail(s, MPM_INVALID_ARG, "nu must lie in (-1, 0.5)");
  if (!(e.dt > 0.f)) return sfail(s, MPM_INVALID_ARG, "dt must be > 0");
  if (r->n_more < 0 || r->n_more > MPM_MAX_COLLIDERS - 1)
    return sfail(s, MPM_INVALID_ARG, "n_more outside [0, MPM_MAX_COLLIDERS - 1]");
  for (int k = 0; k < r->n_more; ++k)
    if (r->more[k].shape < MPM_COLLIDER_BOX || r->more[k].shape > MPM_COLLIDER_ROUNDED_BOX)
      return sfail(s, MPM_INVALID_ARG, "unknown collider shape");
  Req q;
  q.id = s->next_id++;
  q.r = *r;
  q.arrival = r->arrival >= 0.0 ? r->arrival : now_s(s);
  q.nchunks = (int)ceil_div(r->substeps, s->d.chunk);
  q.chunk_len.assign(q.nchunks, 0);
  q.chunk_clock.assign(q.nchunks, 0);
  q.nbytes = resident_bytes(s, *r);
  ++s->submitted;
  if (s->first_arrival < 0.0 || q.arrival < s->first_arrival) s->first_arrival = q.arrival;
  const bool fits = e.n >= 12 && e.n % 4 == 0 && e.n <= s->d.n_cap && e.n_particles <= s->d.n_cap_particles &&
                    e.wall >= 0 && 2 * e.wall + 3 <= e.n && q.nbytes <= s->d.budget_bytes;
  if (!fits) {
    q.state = MPM_REQ_REJECTED;
    q.finished = now_s(s);
    ++s->n_rejected;
  } else {
    s->queue.push_back(q.id);
  }
  *id = q.id;
  s->reqs.emplace(q.id, std::move(q));
  return MPM_OK;
}

int mpm_server_step(mpm_server* s) {
  if (!s) return MPM_INVALID_ARG;
  int rc = admit(s);
  if (rc != MPM_OK) return rc;
  rc = forward_chunk(s);
  if (rc != MPM_OK) return rc;
  std::vector<int64_t> bwd_ids;
  rc = backward_chunk(s, bwd_ids);
  if (rc != MPM_OK) return rc;
  rc = finish_step(s, bwd_ids);
  ++s->steps;
  return rc;
}

int mpm_server_poll(mpm_server* s, int64_t id, mpm_request_status* st) {
  if (!s || !st) return MPM_INVALID_ARG;
  std::memset(st, 0, sizeof(*st));
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) {
    st->state = MPM_REQ_UNKNOWN;
    return MPM_OK;
  }
  const Req& q = it->second;
  st->state = q.state;
  st->error_bits = q.err_bits;
  st->arrival = q.arrival;
  st->admitted = q.admitted;
  st->finished = q.finished;
  for (int k = 0; k < 8; ++k) st->dparams[k] = q.dparams[k];
  if (q.state != MPM_REQ_QUEUED && q.state != MPM_REQ_RUNNING) s->reqs.erase(it);
  return MPM_OK;
}

int mpm_server_cancel(mpm_server* s, int64_t id) {
  if (!s) return MPM_INVALID_ARG;
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return sfail(s, MPM_INVALID_ARG, "no such request");
  Req& q = it->second;
  if (q.state == MPM_REQ_QUEUED) {
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), id));
    q.state = MPM_REQ_CANCELLED;
    q.finished = now_s(s);
    ++s->n_cancelled;
    return MPM_OK;
  }
  if (q.state == MPM_REQ_RUNNING) return release(s, q, MPM_REQ_CANCELLED);
  return sfail(s, MPM_INVALID_ARG, "the request is not queued or running");
}

double mpm_server_now(const mpm_server* s) { return s ? now_s(s) : 0.0; }

int mpm_server_idle(const mpm_server* s) {
  if (!s) return 1;
  if (!s->queue.empty()) return 0;
  for (int64_t id : s->slot_req)
    if (id >= 0) return 0;
  return 1;
}

int mpm_server_stats_get(mpm_server* s, mpm_server_stats* st) {
  if (!s || !st) return MPM_INVALID_ARG;
  std::memset(st, 0, sizeof(*st));
  st->submitted = s->submitted;
  st->done = s->n_done;
  st->errors = s->n_errors;
  st->cancelled = s->n_cancelled;
  st->rejected = s->n_rejected;
  st->queued = (int64_t)s->queue.size();
  for (int64_t id : s->slot_req) st->running += id >= 0;
  st->particle_substeps = s->work;
  st->steps = s->steps;
  st->max_running = s->max_running;
  st->bytes_in_use = s->used;
  st->p50_ms = 1e3 * percentile(s->lat, 50.0);
  st->p99_ms = 1e3 * percentile(s->lat, 99.0);
  st->first_arrival = s->first_arrival < 0.0 ? 0.0 : s->first_arrival;
  st->last_finish = s->last_finish;
  return MPM_OK;
}

const char* mpm_server_last_error(const mpm_server* s) { return s ? s->err.c_str() : "null server"; }

}  // extern "C"
