// Host side of the rigid-body batch (include/mpm_rb.h): validation, the tree's
// ancestor and descendant masks, device memory, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mpm_rb.h"
#include "rb_kernels.h"

struct mpm_rb {
  int E = 0, N = 0, C = 0, max_S = 0;
  float dt = 0.f;
  float g[3] = {0.f, 0.f, 0.f};
  float zref = 0.f;
  hipStream_t stream = nullptr;
  bool has_alloc = false;
  mpm_allocator alloc{};
  std::vector<std::pair<void*, size_t>> allocations;
  int64_t bytes = 0;
  std::string err;

  float* link = nullptr;       // [N][kRbLinkF]
  uint64_t* anc = nullptr;     // [N]
  uint64_t* desc = nullptr;    // [N]
  uint64_t* kids = nullptr;    // [N]
  int32_t* level = nullptr;    // [N] height | depth << 16
  uint64_t* hmask = nullptr;   // [H]
  int H = 0, D = 0;
  int32_t* cbeg = nullptr;     // [N + 1]
  float* contact = nullptr;    // [C][4]
  float* prm = nullptr;        // [E][kRbPrm] FP32 copy of the parameters
  float* q = nullptr;
  float* qd = nullptr;
  float* tape = nullptr;       // [(max_S + 1)][E][2][N]
  float* tape_tau = nullptr;   // [max_S][E][N]
  int32_t* errs = nullptr;
  int recorded = -1;           // substeps of the kept record, -1: none
  std::vector<int32_t> env_err_h;
};

namespace {

int fail(mpm_rb* r, int code, const std::string& msg) {
  if (r) r->err = msg;
  return code;
}

#define RBC(r, expr)                                                                      \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      return fail((r), MPM_DEVICE_ERROR, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

void* ralloc(mpm_rb* r, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  void* p = nullptr;
  if (r->has_alloc) {
    p = r->alloc.alloc(bytes, r->alloc.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) {
    r->allocations.push_back({p, bytes});
    r->bytes += (int64_t)bytes;
  }
  return p;
}

void free_all(mpm_rb* r) {
  for (auto& a : r->allocations) {
    if (r->has_alloc)
      r->alloc.free(a.first, r->alloc.ctx);
    else
      (void)hipFree(a.first);
  }
  r->allocations.clear();
  r->bytes = 0;
}

mpmx::RbModel model_of(const mpm_rb* r) {
  mpmx::RbModel m;
  m.E = r->E;
  m.N = r->N;
  m.C = r->C;
  m.link = r->link;
  m.anc = r->anc;
  m.desc = r->desc;
  m.kids = r->kids;
  m.level = r->level;
  m.hmask = r->hmask;
  m.H = r->H;
  m.D = r->D;
  m.cbeg = r->cbeg;
  m.contact = r->contact;
  m.prm = r->prm;
  m.dt = r->dt;
  for (int a = 0; a < 3; ++a) m.g[a] = r->g[a];
  m.zref = r->zref;
  return m;
}

bool finite_n(const float* p, int n) {
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(p[k])) return false;
  return true;
}

// joint_rot must be a rotation: R R^T = I to 1e-4 and det R > 0
bool is_rotation(const float* R) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += (double)R[3 * i + k] * R[3 * j + k];
      if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-4) return false;
    }
  const double det = (double)R[0] * (R[4] * R[8] - R[5] * R[7]) - (double)R[1] * (R[3] * R[8] - R[5] * R[6]) +
                     (double)R[2] * (R[3] * R[7] - R[4] * R[6]);
  return det > 0.0;
}

}  // namespace

extern "C" {

int mpm_rb_create(const mpm_rb_desc* d, const mpm_rb_link* links, const mpm_rb_contact* contacts,
                  const mpm_allocator* alloc, void* stream, mpm_rb** out) {
  if (!d || !links || !out) return MPM_INVALID_ARG;
  *out = nullptr;
  if (d->n_envs < 1 || d->n_links < 1 || d->n_links > MPM_RB_MAX_LINKS || d->n_contacts < 0 ||
      d->n_contacts > MPM_RB_MAX_CONTACTS || (d->n_contacts > 0 && !contacts) || d->max_substeps < 0 ||
      !(d->dt > 0.f) || !std::isfinite(d->dt) || !finite_n(d->gravity, 3))
    return MPM_INVALID_ARG;
  if (alloc && (!alloc->alloc || !alloc->free)) return MPM_INVALID_ARG;
  const int N = d->n_links, C = d->n_contacts;
  // links: order, finiteness, rotations, unit axes; masks of root paths and subtrees
  std::vector<float> lk((size_t)N * mpmx::kRbLinkF);
  std::vector<uint64_t> anc(N, 0), desc(N, 0);
  if (links[0].parent != -1) return MPM_INVALID_ARG;
  const float ref[3] = {links[0].joint_pos[0], links[0].joint_pos[1], links[0].joint_pos[2]};
  for (int i = 0; i < N; ++i) {
    const mpm_rb_link& L = links[i];
    if (L.parent < -1 || L.parent >= i) return MPM_INVALID_ARG;
    if (!finite_n(L.joint_rot, 9) || !finite_n(L.joint_pos, 3) || !finite_n(L.axis, 3) || !std::isfinite(L.mass) ||
        !finite_n(L.com, 3) || !finite_n(L.inertia, 6) || L.mass < 0.f || !is_rotation(L.joint_rot) ||
        (L.joint != MPM_RB_REVOLUTE && L.joint != MPM_RB_PRISMATIC))
      return MPM_INVALID_ARG;
    const double an = std::sqrt((double)L.axis[0] * L.axis[0] + (double)L.axis[1] * L.axis[1] +
                                (double)L.axis[2] * L.axis[2]);
    if (std::fabs(an - 1.0) > 1e-4) return MPM_INVALID_ARG;
    float* row = &lk[(size_t)i * mpmx::kRbLinkF];
    std::memcpy(row, L.joint_rot, 9 * sizeof(float));
    for (int a = 0; a < 3; ++a) {
      // the spatial origin is link 0's joint origin (smaller lever arms keep FP32 inertias about it accurate)
      row[9 + a] = L.parent < 0 ? L.joint_pos[a] - ref[a] : L.joint_pos[a];
      row[12 + a] = (float)(L.axis[a] / an);
      row[16 + a] = L.com[a];
    }
    row[15] = L.mass;
    std::memcpy(row + 19, L.inertia, 6 * sizeof(float));
    row[25] = L.joint == MPM_RB_PRISMATIC ? 1.f : 0.f;
    anc[i] = (L.parent >= 0 ? anc[L.parent] : 0ull) | (1ull << i);
  }
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < N; ++k)
      if (anc[k] & (1ull << i)) desc[i] |= 1ull << k;
  // levels: depth = joints above the link, height = longest path down to a leaf (children have higher indices)
  std::vector<int32_t> depth(N, 0), height(N, 0), level(N);
  int H = 1, D = 1;
  for (int i = 0; i < N; ++i) depth[i] = links[i].parent < 0 ? 0 : depth[links[i].parent] + 1;
  for (int i = N - 1; i >= 0; --i)
    if (links[i].parent >= 0) height[links[i].parent] = std::max(height[links[i].parent], height[i] + 1);
  std::vector<uint64_t> hmask(N, 0), kids(N, 0);
  for (int i = 0; i < N; ++i)
    if (links[i].parent >= 0) kids[links[i].parent] |= 1ull << i;
  for (int i = 0; i < N; ++i) {
    level[i] = height[i] | (depth[i] << 16);
    hmask[height[i]] |= 1ull << i;
    H = std::max(H, height[i] + 1);
    D = std::max(D, depth[i] + 1);
  }
  // contacts grouped by link
  std::vector<int32_t> cbeg(N + 1, 0);
  for (int c = 0; c < C; ++c) {
    const mpm_rb_contact& K = contacts[c];
    if (K.link < 0 || K.link >= N || !finite_n(K.centre, 3) || !std::isfinite(K.radius) || K.radius < 0.f)
      return MPM_INVALID_ARG;
    ++cbeg[K.link + 1];
  }
  for (int i = 0; i < N; ++i) cbeg[i + 1] += cbeg[i];
  std::vector<float> ct((size_t)(C > 0 ? C : 1) * 4, 0.f);
  {
    std::vector<int32_t> fill(cbeg.begin(), cbeg.end() - 1);
    for (int c = 0; c < C; ++c) {
      const mpm_rb_contact& K = contacts[c];
      float* row = &ct[(size_t)fill[K.link]++ * 4];
      row[0] = K.centre[0];
      row[1] = K.centre[1];
      row[2] = K.centre[2];
      row[3] = K.radius;
    }
  }

  mpm_rb* r = new mpm_rb();
  r->E = d->n_envs;
  r->N = N;
  r->C = C;
  r->max_S = d->max_substeps;
  r->dt = d->dt;
  for (int a = 0; a < 3; ++a) r->g[a] = d->gravity[a];
  r->zref = ref[2];
  r->H = H;
  r->D = D;
  r->stream = (hipStream_t)stream;
  if (alloc) {
    r->has_alloc = true;
    r->alloc = *alloc;
  }
  const size_t E = r->E;
  r->link = (float*)ralloc(r, sizeof(float) * lk.size());
  r->anc = (uint64_t*)ralloc(r, sizeof(uint64_t) * N);
  r->desc = (uint64_t*)ralloc(r, sizeof(uint64_t) * N);
  r->cbeg = (int32_t*)ralloc(r, sizeof(int32_t) * (N + 1));
  r->level = (int32_t*)ralloc(r, sizeof(int32_t) * N);
  r->kids = (uint64_t*)ralloc(r, sizeof(uint64_t) * N);
  r->hmask = (uint64_t*)ralloc(r, sizeof(uint64_t) * N);
  r->contact = (float*)ralloc(r, sizeof(float) * ct.size());
  r->prm = (float*)ralloc(r, sizeof(float) * mpmx::kRbPrm * E);
  r->q = (float*)ralloc(r, sizeof(float) * E * N);
  r->qd = (float*)ralloc(r, sizeof(float) * E * N);
  r->tape = (float*)ralloc(r, sizeof(float) * 2 * E * N * (size_t)(r->max_S + 1));
  r->tape_tau = (float*)ralloc(r, sizeof(float) * E * N * (size_t)(r->max_S > 0 ? r->max_S : 1));
  r->errs = (int32_t*)ralloc(r, sizeof(int32_t) * E);
  if (!(r->link && r->anc && r->desc && r->kids && r->level && r->hmask && r->cbeg && r->contact && r->prm && r->q && r->qd && r->tape && r->tape_tau &&
        r->errs)) {
    free_all(r);
    delete r;
    return MPM_OUT_OF_MEMORY;
  }
  r->env_err_h.assign(E, 0);
  std::vector<float> prm(mpmx::kRbPrm * E);
  for (size_t e = 0; e < E; ++e) {
    const float row[mpmx::kRbPrm] = {0.f, 0.f, 0.f, 0.f, -INFINITY};
    std::memcpy(&prm[mpmx::kRbPrm * e], row, sizeof row);
  }
  hipError_t e1 = hipMemcpyAsync(r->link, lk.data(), sizeof(float) * lk.size(), hipMemcpyHostToDevice, r->stream);
  if (e1 == hipSuccess) e1 = hipMemcpyAsync(r->anc, anc.data(), sizeof(uint64_t) * N, hipMemcpyHostToDevice, r->stream);
  if (e1 == hipSuccess) e1 = hipMemcpyAsync(r->desc, desc.data(), sizeof(uint64_t) * N, hipMemcpyHostToDevice, r->stream);
  if (e1 == hipSuccess) e1 = hipMemcpyAsync(r->kids, kids.data(), sizeof(uint64_t) * N, hipMemcpyHostToDevice, r->stream);
  if (e1 == hipSuccess) e1 = hipMemcpyAsync(r->level, level.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, r->stream);
  if (e1 == hipSuccess) e1 = hipMemcpyAsync(r->hmask, hmask.data(), sizeof(uint64_t) * N, hipMemcpyHostToDevice, r->stream);
  if (e1 == hipSuccess) e1 = hipMemcpyAsync(r->cbeg, cbeg.data(), sizeof(int32_t) * (N + 1), hipMemcpyHostToDevice, r->stream);
  if (e1 == hipSuccess) e1 = hipMemcpyAsync(r->contact, ct.data(), sizeof(float) * ct.size(), hipMemcpyHostToDevice, r->stream);
  if (e1 == hipSuccess) e1 = hipMemcpyAsync(r->prm, prm.data(), sizeof(float) * prm.size(), hipMemcpyHostToDevice, r->stream);
  if (e1 == hipSuccess) e1 = hipMemsetAsync(r->q, 0, sizeof(float) * E * N, r->stream);
  if (e1 == hipSuccess) e1 = hipMemsetAsync(r->qd, 0, sizeof(float) * E * N, r->stream);
  if (e1 == hipSuccess) e1 = hipMemsetAsync(r->errs, 0, sizeof(int32_t) * E, r->stream);
  if (e1 == hipSuccess) e1 = hipStreamSynchronize(r->stream);
  if (e1 != hipSuccess) {
    free_all(r);
    delete r;
    return MPM_DEVICE_ERROR;
  }
  *out = r;
  return MPM_OK;
}

int mpm_rb_destroy(mpm_rb* r) {
  if (!r) return MPM_INVALID_ARG;
  (void)hipStreamSynchronize(r->stream);
  free_all(r);
  delete r;
  return MPM_OK;
}

int mpm_rb_set_params(mpm_rb* r, const double* params) {
  if (!r) return MPM_INVALID_ARG;
  if (!params) return fail(r, MPM_INVALID_ARG, "null parameters");
  std::vector<float> p(mpmx::kRbPrm * (size_t)r->E);
  for (int e = 0; e < r->E; ++e) {
    const double* w = params + mpmx::kRbPrm * (size_t)e;
    bool ok = std::isfinite(w[0]) && std::isfinite(w[1]) && std::isfinite(w[2]) && std::isfinite(w[3]) &&
              !std::isnan(w[4]) && w[4] != INFINITY;
    ok = ok && w[0] >= 0.0 && w[1] >= 0.0 && w[2] >= 0.0 && w[3] >= 0.0;
    if (!ok) return fail(r, MPM_INVALID_ARG, "parameters of env " + std::to_string(e) + " out of range");
    for (int c = 0; c < mpmx::kRbPrm; ++c) p[mpmx::kRbPrm * (size_t)e + c] = (float)w[c];
  }
  RBC(r, hipMemcpyAsync(r->prm, p.data(), sizeof(float) * p.size(), hipMemcpyHostToDevice, r->stream));
  RBC(r, hipStreamSynchronize(r->stream));   // p is a host temporary
  r->recorded = -1;
  return MPM_OK;
}

int mpm_rb_set_state(mpm_rb* r, const float* q, const float* qd) {
  if (!r) return MPM_INVALID_ARG;
  if (!q) return fail(r, MPM_INVALID_ARG, "null joint angles");
  const size_t nb = sizeof(float) * (size_t)r->E * r->N;
  RBC(r, hipMemcpyAsync(r->q, q, nb, hipMemcpyDeviceToDevice, r->stream));
  if (qd)
    RBC(r, hipMemcpyAsync(r->qd, qd, nb, hipMemcpyDeviceToDevice, r->stream));
  else
    RBC(r, hipMemsetAsync(r->qd, 0, nb, r->stream));
  r->recorded = -1;
  return MPM_OK;
}

int mpm_rb_get_state(mpm_rb* r, float* q, float* qd) {
  if (!r) return MPM_INVALID_ARG;
  const size_t nb = sizeof(float) * (size_t)r->E * r->N;
  if (q) RBC(r, hipMemcpyAsync(q, r->q, nb, hipMemcpyDeviceToDevice, r->stream));
  if (qd) RBC(r, hipMemcpyAsync(qd, r->qd, nb, hipMemcpyDeviceToDevice, r->stream));
  return MPM_OK;
}

int mpm_rb_forward(mpm_rb* r, int32_t S, const float* tau, int32_t flags) {
  if (!r) return MPM_INVALID_ARG;
  if (S < 0) return fail(r, MPM_INVALID_ARG, "negative substep count");
  const bool record = (flags & MPM_FWD_RECORD) != 0;
  if (record && S > r->max_S) return fail(r, MPM_BAD_STATE, "record longer than the tape (max_substeps)");
  r->recorded = -1;
  mpmx::launch_rb_forward(model_of(r), S, r->q, r->qd, tau, record ? r->tape : nullptr,
                          record ? r->tape_tau : nullptr, r->errs, r->stream);
  RBC(r, hipGetLastError());
  if (record) r->recorded = S;
  return MPM_OK;
}

int mpm_rb_backward(mpm_rb* r, const float* gq, const float* gqd, float* dq0, float* dqd0, float* dtau,
                    double* dparams) {
  if (!r) return MPM_INVALID_ARG;
  if (!dq0 || !dqd0) return fail(r, MPM_INVALID_ARG, "null output cotangents");
  if (r->recorded < 0) return fail(r, MPM_BAD_STATE, "no recorded forward");
  mpmx::launch_rb_backward(model_of(r), r->recorded, r->tape, r->tape_tau, gq, gqd, dq0, dqd0, dtau, dparams,
                           r->stream);
  RBC(r, hipGetLastError());
  return MPM_OK;
}

int mpm_rb_sync(mpm_rb* r) {
  if (!r) return MPM_INVALID_ARG;
  RBC(r, hipStreamSynchronize(r->stream));
  RBC(r, hipMemcpy(r->env_err_h.data(), r->errs, sizeof(int32_t) * r->E, hipMemcpyDeviceToHost));
  int agg = 0;
  for (int v : r->env_err_h) agg |= v;
  if (agg) {
    RBC(r, hipMemsetAsync(r->errs, 0, sizeof(int32_t) * r->E, r->stream));
    RBC(r, hipStreamSynchronize(r->stream));
    return fail(r, MPM_NONFINITE, "non-finite rigid-body state");
  }
  return MPM_OK;
}

int mpm_rb_env_errors(mpm_rb* r, int32_t* errs) {
  if (!r || !errs) return MPM_INVALID_ARG;
  std::memcpy(errs, r->env_err_h.data(), sizeof(int32_t) * r->E);
  return MPM_OK;
}

const char* mpm_rb_last_error(const mpm_rb* r) {
  if (!r) return "null rigid-body batch";
  return r->err.c_str();
}

int64_t mpm_rb_memory_bytes(const mpm_rb* r) { return r ? r->bytes : 0; }

}  // extern "C"
