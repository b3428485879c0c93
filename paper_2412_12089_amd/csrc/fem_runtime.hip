// Host side of the FEM batch (include/mpm_fem.h): validation, device memory,
// the node -> element incidences of the shared topology, launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mpm_fem.h"
#include "fem_kernels.h"

struct mpm_fem {
  int E = 0, n = 0, T = 0, max_S = 0;
  float dt = 0.f;
  float g[3] = {0.f, 0.f, 0.f};
  hipStream_t stream = nullptr;
  bool has_alloc = false;
  mpm_allocator alloc{};
  std::vector<std::pair<void*, size_t>> allocations;
  int64_t bytes = 0;
  std::string err;

  int4* tets = nullptr;
  int32_t* inc_off = nullptr;
  int32_t* inc = nullptr;
  float* Bm[2] = {nullptr, nullptr};   // rest data is double-buffered: a degenerate mesh leaves the old one
  float* W[2] = {nullptr, nullptr};
  float* wm[2] = {nullptr, nullptr};
  int cur = 0;
  bool has_rest = false;
  float* prm = nullptr;                 // [E][8] FP32 copy of the parameters
  float* x = nullptr;
  float* v = nullptr;
  float* tape = nullptr;                // [(max_S + 1)][E][n][6]
  float* tape_act = nullptr;            // [max_S][E][T]
  int32_t* errs = nullptr;
  int32_t* bad = nullptr;
  int recorded = -1;                    // substeps of the kept record, -1: none
  std::vector<int32_t> env_err_h;
};

namespace {

int fail(mpm_fem* f, int code, const std::string& msg) {
  if (f) f->err = msg;
  return code;
}

#define FEMC(f, expr)                                                                     \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      return fail((f), MPM_DEVICE_ERROR, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

void* falloc(mpm_fem* f, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  void* p = nullptr;
  if (f->has_alloc) {
    p = f->alloc.alloc(bytes, f->alloc.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) {
    f->allocations.push_back({p, bytes});
    f->bytes += (int64_t)bytes;
  }
  return p;
}

void free_all(mpm_fem* f) {
  for (auto& a : f->allocations) {
    if (f->has_alloc)
      f->alloc.free(a.first, f->alloc.ctx);
    else
      (void)hipFree(a.first);
  }
  f->allocations.clear();
  f->bytes = 0;
}

mpmx::FemMesh mesh_of(const mpm_fem* f) {
  mpmx::FemMesh m;
  m.E = f->E;
  m.n = f->n;
  m.T = f->T;
  m.tets = f->tets;
  m.inc_off = f->inc_off;
  m.inc = f->inc;
  m.Bm = f->Bm[f->cur];
  m.W = f->W[f->cur];
  m.wm = f->wm[f->cur];
  m.prm = f->prm;
  m.dt = f->dt;
  for (int a = 0; a < 3; ++a) m.g[a] = f->g[a];
  return m;
}

bool finite_prm(const double* p) {
  for (int c = 0; c < MPM_FEM_PARAMS; ++c)
    if (c != 7 && !std::isfinite(p[c])) return false;
  return !std::isnan(p[7]);
}

}  // namespace

extern "C" {

int mpm_fem_create(const mpm_fem_desc* d, const int32_t* tets, const mpm_allocator* alloc, void* stream,
                   mpm_fem** out) {
  if (!d || !tets || !out) return MPM_INVALID_ARG;
  *out = nullptr;
  if (d->n_envs < 1 || d->n_nodes < 4 || d->n_nodes > MPM_FEM_MAX_NODES || d->n_tets < 1 ||
      d->n_tets > MPM_FEM_MAX_TETS || d->max_substeps < 0 || !(d->dt > 0.f) || !std::isfinite(d->dt))
    return MPM_INVALID_ARG;
  if (alloc && (!alloc->alloc || !alloc->free)) return MPM_INVALID_ARG;
  const int n = d->n_nodes, T = d->n_tets;
  // topology and the node -> (element, corner) incidences
  std::vector<int> count(n + 1, 0);
  for (int t = 0; t < T; ++t) {
    const int32_t* q = tets + 4 * t;
    for (int c = 0; c < 4; ++c) {
      if (q[c] < 0 || q[c] >= n) return MPM_INVALID_ARG;
      for (int c2 = 0; c2 < c; ++c2)
        if (q[c2] == q[c]) return MPM_INVALID_ARG;
      ++count[q[c] + 1];
    }
  }
  for (int i = 0; i < n; ++i)
    if (count[i + 1] == 0) return MPM_INVALID_ARG;   // a node in no element would have no mass
  std::vector<int32_t> off(n + 1, 0), inc(4 * (size_t)T);
  for (int i = 0; i < n; ++i) off[i + 1] = off[i] + count[i + 1];
  std::vector<int> fill(off.begin(), off.end() - 1);
  for (int t = 0; t < T; ++t)
    for (int c = 0; c < 4; ++c) inc[fill[tets[4 * t + c]]++] = t * 4 + c;

  mpm_fem* f = new mpm_fem();
  f->E = d->n_envs;
  f->n = n;
  f->T = T;
  f->max_S = d->max_substeps;
  f->dt = d->dt;
  for (int a = 0; a < 3; ++a) f->g[a] = d->gravity[a];
  f->stream = (hipStream_t)stream;
  if (alloc) {
    f->has_alloc = true;
    f->alloc = *alloc;
  }
  const size_t E = f->E;
  f->tets = (int4*)falloc(f, sizeof(int4) * T);
  f->inc_off = (int32_t*)falloc(f, sizeof(int32_t) * (n + 1));
  f->inc = (int32_t*)falloc(f, sizeof(int32_t) * 4 * T);
  for (int b = 0; b < 2; ++b) {
    f->Bm[b] = (float*)falloc(f, sizeof(float) * 9 * E * T);
    f->W[b] = (float*)falloc(f, sizeof(float) * E * T);
    f->wm[b] = (float*)falloc(f, sizeof(float) * E * n);
  }
  f->prm = (float*)falloc(f, sizeof(float) * MPM_FEM_PARAMS * E);
  f->x = (float*)falloc(f, sizeof(float) * 3 * E * n);
  f->v = (float*)falloc(f, sizeof(float) * 3 * E * n);
  f->tape = (float*)falloc(f, sizeof(float) * 6 * E * n * (size_t)(f->max_S + 1));
  f->tape_act = (float*)falloc(f, sizeof(float) * E * T * (size_t)(f->max_S > 0 ? f->max_S : 1));
  f->errs = (int32_t*)falloc(f, sizeof(int32_t) * E);
  f->bad = (int32_t*)falloc(f, sizeof(int32_t));
  bool ok = f->tets && f->inc_off && f->inc && f->prm && f->x && f->v && f->tape && f->tape_act && f->errs && f->bad;
  for (int b = 0; b < 2; ++b) ok = ok && f->Bm[b] && f->W[b] && f->wm[b];
  if (!ok) {
    free_all(f);
    delete f;
    return MPM_OUT_OF_MEMORY;
  }
  f->env_err_h.assign(E, 0);
  std::vector<float> prm(MPM_FEM_PARAMS * E);
  for (size_t e = 0; e < E; ++e) {
    const float row[MPM_FEM_PARAMS] = {1.f, 1.f, 1.f, 0.f, 0.f, 0.f, 0.f, -INFINITY};
    std::memcpy(&prm[MPM_FEM_PARAMS * e], row, sizeof row);
  }
  hipError_t e1 = hipMemcpyAsync(f->tets, tets, sizeof(int4) * T, hipMemcpyHostToDevice, f->stream);
  if (e1 == hipSuccess) e1 = hipMemcpyAsync(f->inc_off, off.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, f->stream);
  if (e1 == hipSuccess) e1 = hipMemcpyAsync(f->inc, inc.data(), sizeof(int32_t) * 4 * T, hipMemcpyHostToDevice, f->stream);
  if (e1 == hipSuccess) e1 = hipMemcpyAsync(f->prm, prm.data(), sizeof(float) * prm.size(), hipMemcpyHostToDevice, f->stream);
  if (e1 == hipSuccess) e1 = hipMemsetAsync(f->x, 0, sizeof(float) * 3 * E * n, f->stream);
  if (e1 == hipSuccess) e1 = hipMemsetAsync(f->v, 0, sizeof(float) * 3 * E * n, f->stream);
  if (e1 == hipSuccess) e1 = hipMemsetAsync(f->errs, 0, sizeof(int32_t) * E, f->stream);
  if (e1 == hipSuccess) e1 = hipStreamSynchronize(f->stream);
  if (e1 != hipSuccess) {
    free_all(f);
    delete f;
    return MPM_DEVICE_ERROR;
  }
  *out = f;
  return MPM_OK;
}

int mpm_fem_destroy(mpm_fem* f) {
  if (!f) return MPM_INVALID_ARG;
  (void)hipStreamSynchronize(f->stream);
  free_all(f);
  delete f;
  return MPM_OK;
}

int mpm_fem_set_rest(mpm_fem* f, const float* X) {
  if (!f) return MPM_INVALID_ARG;
  if (!X) return fail(f, MPM_INVALID_ARG, "null rest positions");
  const int nb = 1 - f->cur;
  mpmx::FemMesh m = mesh_of(f);
  FEMC(f, hipMemsetAsync(f->bad, 0, sizeof(int32_t), f->stream));
  mpmx::launch_fem_rest(m, X, f->Bm[nb], f->W[nb], f->wm[nb], f->bad, f->stream);
  FEMC(f, hipGetLastError());
  int32_t bad = 0;
  FEMC(f, hipMemcpyAsync(&bad, f->bad, sizeof(int32_t), hipMemcpyDeviceToHost, f->stream));
  FEMC(f, hipStreamSynchronize(f->stream));
  if (bad) return fail(f, MPM_BAD_STATE, "degenerate element in the rest shape");
  f->cur = nb;
  f->has_rest = true;
  f->recorded = -1;
  return MPM_OK;
}

int mpm_fem_set_params(mpm_fem* f, const double* params) {
  if (!f) return MPM_INVALID_ARG;
  if (!params) return fail(f, MPM_INVALID_ARG, "null parameters");
  std::vector<float> p(MPM_FEM_PARAMS * (size_t)f->E);
  for (int e = 0; e < f->E; ++e) {
    const double* r = params + MPM_FEM_PARAMS * (size_t)e;
    if (!finite_prm(r) || !(r[1] > 0.0) || !(r[2] > 0.0) || r[3] < 0.0 || r[4] < 0.0 || r[5] < 0.0 || r[6] < 0.0)
      return fail(f, MPM_INVALID_ARG, "parameters of env " + std::to_string(e) + " out of range");
    for (int c = 0; c < MPM_FEM_PARAMS; ++c) p[MPM_FEM_PARAMS * (size_t)e + c] = (float)r[c];
  }
  FEMC(f, hipMemcpyAsync(f->prm, p.data(), sizeof(float) * p.size(), hipMemcpyHostToDevice, f->stream));
  FEMC(f, hipStreamSynchronize(f->stream));   // p is a host temporary
  f->recorded = -1;
  return MPM_OK;
}

int mpm_fem_set_state(mpm_fem* f, const float* x, const float* v) {
  if (!f) return MPM_INVALID_ARG;
  if (!x) return fail(f, MPM_INVALID_ARG, "null positions");
  const size_t nb = sizeof(float) * 3 * (size_t)f->E * f->n;
  FEMC(f, hipMemcpyAsync(f->x, x, nb, hipMemcpyDeviceToDevice, f->stream));
  if (v)
    FEMC(f, hipMemcpyAsync(f->v, v, nb, hipMemcpyDeviceToDevice, f->stream));
  else
    FEMC(f, hipMemsetAsync(f->v, 0, nb, f->stream));
  f->recorded = -1;
  return MPM_OK;
}

int mpm_fem_get_state(mpm_fem* f, float* x, float* v) {
  if (!f) return MPM_INVALID_ARG;
  const size_t nb = sizeof(float) * 3 * (size_t)f->E * f->n;
  if (x) FEMC(f, hipMemcpyAsync(x, f->x, nb, hipMemcpyDeviceToDevice, f->stream));
  if (v) FEMC(f, hipMemcpyAsync(v, f->v, nb, hipMemcpyDeviceToDevice, f->stream));
  return MPM_OK;
}

int mpm_fem_forward(mpm_fem* f, int32_t S, const float* act, int32_t flags) {
  if (!f) return MPM_INVALID_ARG;
  if (S < 0) return fail(f, MPM_INVALID_ARG, "negative substep count");
  if (!f->has_rest) return fail(f, MPM_BAD_STATE, "no rest shape set");
  const bool record = (flags & MPM_FWD_RECORD) != 0;
  if (record && S > f->max_S) return fail(f, MPM_BAD_STATE, "record longer than the tape (max_substeps)");
  f->recorded = -1;
  mpmx::launch_fem_forward(mesh_of(f), S, f->x, f->v, act, record ? f->tape : nullptr,
                           record ? f->tape_act : nullptr, f->errs, f->stream);
  FEMC(f, hipGetLastError());
  if (record) f->recorded = S;
  return MPM_OK;
}

int mpm_fem_backward(mpm_fem* f, const float* gx, const float* gv, float* dx0, float* dv0, float* dact,
                     double* dparams) {
  if (!f) return MPM_INVALID_ARG;
  if (!dx0 || !dv0) return fail(f, MPM_INVALID_ARG, "null output cotangents");
  if (f->recorded < 0) return fail(f, MPM_BAD_STATE, "no recorded forward");
  mpmx::launch_fem_backward(mesh_of(f), f->recorded, f->tape, f->tape_act, gx, gv, dx0, dv0, dact, dparams,
                            f->stream);
  FEMC(f, hipGetLastError());
  return MPM_OK;
}

int mpm_fem_sync(mpm_fem* f) {
  if (!f) return MPM_INVALID_ARG;
  FEMC(f, hipStreamSynchronize(f->stream));
  FEMC(f, hipMemcpy(f->env_err_h.data(), f->errs, sizeof(int32_t) * f->E, hipMemcpyDeviceToHost));
  int agg = 0;
  for (int v : f->env_err_h) agg |= v;
  if (agg) {
    FEMC(f, hipMemsetAsync(f->errs, 0, sizeof(int32_t) * f->E, f->stream));
    FEMC(f, hipStreamSynchronize(f->stream));
    return fail(f, MPM_NONFINITE, "non-finite FEM state");
  }
  return MPM_OK;
}

int mpm_fem_env_errors(mpm_fem* f, int32_t* errs) {
  if (!f || !errs) return MPM_INVALID_ARG;
  std::memcpy(errs, f->env_err_h.data(), sizeof(int32_t) * f->E);
  return MPM_OK;
}

const char* mpm_fem_last_error(const mpm_fem* f) {
  if (!f) return "null FEM batch";
  return f->err.c_str();
}

int64_t mpm_fem_memory_bytes(const mpm_fem* f) { return f ? f->bytes : 0; }

}  // extern "C"
