// Host library: the C ABI of include/mf.h.  Validation, handle lifetime,
// workspace layout and kernel dispatch.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "mf.h"
#include "mf_internal.h"

struct mf_handle {
  mf_desc d;
  hipStream_t stream = nullptr;
  mf::WorkspaceLayout ws;
  int cur = 0;      // state buffer holding the current iterate
  int iter = 0;     // steps since (re)initialisation
  int k_launch = 1; // steps fused per launch
  std::string err;
};

namespace {

thread_local std::string g_err;

mf_status fail(mf_handle* h, mf_status st, const std::string& msg) {
  if (h) h->err = msg;
  g_err = msg;
  return st;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool is_grid(int g) { return g == MF_GRID4 || g == MF_GRID8; }

mf::WorkspaceLayout layout_for(const mf_desc& d) {
  mf::WorkspaceLayout w;
  size_t off = 0;
  w.flags = off;
  off += 256;
  w.n_blocks = mf::grid_blocks_per_item(1, d.n_nodes);
  w.partials = off;
  off += align256(sizeof(double) * (size_t)d.batch * (size_t)w.n_blocks);
  w.f_out = off;
  off += align256(sizeof(double) * (size_t)d.batch);
  w.total = off;
  return w;
}

// Every rule checked before anything is enqueued.
mf_status check_desc(const mf_desc* d, std::string* msg) {
  auto bad = [&](const char* m) { *msg = m; return MF_EINVAL; };
  if (!d) return bad("descriptor is NULL");
  if (d->abi_version != MF_ABI_VERSION) return bad("abi_version mismatch");
  if (d->batch < 1) return bad("batch must be >= 1");
  if (d->n_nodes < 1) return bad("n_nodes must be >= 1");
  if (d->n_labels < 1) return bad("n_labels must be >= 1");
  if (!(d->alpha > 0.0 && d->alpha <= 1.0)) return bad("alpha must lie in (0, 1]");
  if (d->graph < MF_GRID4 || d->graph > MF_DENSE) return bad("unknown graph kind");
  if (d->compat != MF_COMPAT_GENERAL && d->compat != MF_COMPAT_POTTS) return bad("unknown compat kind");
  if (d->precision < MF_P_F32 || d->precision > MF_P_F16MSG) return bad("unknown precision");
  if (d->init < MF_INIT_UNARY || d->init > MF_INIT_STATE) return bad("unknown init mode");
  if (!std::isfinite(d->potts_w)) return bad("potts_w must be finite");
  if (is_grid(d->graph)) {
    if (d->height < 1 || d->width < 1) return bad("grid height and width must be >= 1");
    if ((int64_t)d->height * (int64_t)d->width != (int64_t)d->n_nodes) return bad("height * width != n_nodes");
  }
  if (!d->unary) return bad("unary is NULL");
  if (!d->state) return bad("state is NULL");
  if (d->compat == MF_COMPAT_GENERAL && !d->theta) return bad("theta is NULL for a general compatibility");
  if (((uintptr_t)d->unary | (uintptr_t)d->state | (uintptr_t)d->theta) & 3u)
    return bad("float arrays must be 4-byte aligned");
  const size_t elems = (size_t)d->batch * (size_t)d->n_labels * (size_t)d->n_nodes;
  if (elems > ((size_t)1 << 40)) return bad("problem too large");
  const char* s0 = (const char*)d->state;
  const char* s1 = s0 + elems * sizeof(float);
  const char* u0 = (const char*)d->unary;
  const char* u1 = u0 + elems * sizeof(float);
  if (u0 < s0 + 2 * elems * sizeof(float) && s0 < u1) return bad("state overlaps unary");
  (void)s1;
  if (d->n_labels > MF_MAX_LABELS) {
    *msg = "n_labels above MF_MAX_LABELS";
    return MF_EUNSUPPORTED;
  }
  if (!is_grid(d->graph)) {
    *msg = "graph kind not available in this build";
    return MF_EUNSUPPORTED;
  }
  const size_t need = layout_for(*d).total;
  if (!d->workspace || d->workspace_bytes < need) {
    *msg = "workspace missing or smaller than mf_workspace_size";
    return MF_ENOWORKSPACE;
  }
  if ((uintptr_t)d->workspace & 255u) return bad("workspace must be 256-byte aligned");
  return MF_OK;
}

float* buf(const mf_handle* h, int which) {
  const size_t elems = (size_t)h->d.batch * h->d.n_labels * h->d.n_nodes;
  return h->d.state + (size_t)which * elems;
}

int* flags_ptr(const mf_handle* h) { return (int*)((char*)h->d.workspace + h->ws.flags); }

mf_status enqueue_init(mf_handle* h) {
  const mf_desc& d = h->d;
  hipError_t e = mf::launch_clear_flags(flags_ptr(h), 64, h->stream);
  if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("flag clear: ") + hipGetErrorString(e));
  e = mf::launch_init(d.unary, buf(h, 0), d.batch, d.n_labels, d.n_nodes, d.init, flags_ptr(h), h->stream);
  if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("init launch: ") + hipGetErrorString(e));
  h->cur = 0;
  h->iter = 0;
  return MF_OK;
}

// Steps per launch: small grids (fewer 64 x 4 tiles than a few per compute
// unit) are bound by launch and memory latency, so several steps are fused;
// large grids stream HBM at one step per launch.
int choose_steps_per_launch(const mf_desc& d) {
  if (!is_grid(d.graph)) return 1;
  const int kmax = mf::grid_max_steps_per_launch(d.n_labels, d.precision);
  int k = d.steps_per_launch;
  if (k <= 0) {
    const int64_t tiles = (int64_t)d.batch * ((d.width + mf::kTileX - 1) / mf::kTileX) *
                          ((d.height + mf::kTileY - 1) / mf::kTileY);
    k = tiles >= 4 * 256 ? 1 : kmax;
  }
  return k < kmax ? k : kmax;
}

mf_status enqueue_steps(mf_handle* h, int n) {
  const mf_desc& d = h->d;
  while (n > 0) {
    const int ks = n < h->k_launch ? n : h->k_launch;
    mf::StepArgs a;
    a.unary = d.unary;
    a.state_in = buf(h, h->cur);
    a.state_out = buf(h, h->cur ^ 1);
    a.theta = d.theta;
    a.B = d.batch;
    a.L = d.n_labels;
    a.N = d.n_nodes;
    a.H = d.height;
    a.W = d.width;
    a.alpha = (float)d.alpha;
    a.potts_w = d.potts_w;
    const int conn = d.graph == MF_GRID4 ? 4 : 8;
    hipError_t e = ks == 1 ? mf::launch_grid_step(a, conn, d.compat, d.precision, h->stream)
                           : mf::launch_grid_multi_step(a, conn, d.compat, d.precision, h->k_launch, ks,
                                                        h->stream);
    if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
    h->cur ^= 1;
    h->iter += ks;
    n -= ks;
  }
  return MF_OK;
}

}  // namespace

extern "C" {

int32_t mf_abi_version(void) { return MF_ABI_VERSION; }

size_t mf_desc_size(void) { return sizeof(mf_desc); }

size_t mf_workspace_size(const mf_desc* d) {
  if (!d || d->batch < 1 || d->n_nodes < 1 || d->n_labels < 1) return 0;
  return layout_for(*d).total;
}

mf_status mf_validate(const mf_desc* d) {
  std::string msg;
  const mf_status st = check_desc(d, &msg);
  if (st != MF_OK) g_err = msg;
  return st;
}

mf_status mf_init(const mf_desc* d, mf_handle** out) {
  if (!out) return fail(nullptr, MF_EINVAL, "out is NULL");
  *out = nullptr;
  std::string msg;
  const mf_status st = check_desc(d, &msg);
  if (st != MF_OK) return fail(nullptr, st, msg);
  mf_handle* h = new (std::nothrow) mf_handle();
  if (!h) return fail(nullptr, MF_EDEVICE, "host allocation failed");
  h->d = *d;
  h->stream = (hipStream_t)d->stream;
  h->ws = layout_for(*d);
  h->k_launch = choose_steps_per_launch(*d);
  const mf_status s2 = enqueue_init(h);
  if (s2 != MF_OK) {
    g_err = h->err;
    delete h;
    return s2;
  }
  *out = h;
  return MF_OK;
}

mf_status mf_step(mf_handle* h, int32_t n_steps) {
  if (!h) return fail(nullptr, MF_EINVAL, "handle is NULL");
  if (n_steps < 0) return fail(h, MF_EINVAL, "n_steps must be >= 0");
  return enqueue_steps(h, n_steps);
}

mf_status mf_solve(mf_handle* h, int32_t iters, float* q_out) {
  if (!h) return fail(nullptr, MF_EINVAL, "handle is NULL");
  if (iters < 0) return fail(h, MF_EINVAL, "iters must be >= 0");
  if (((uintptr_t)q_out) & 3u) return fail(h, MF_EINVAL, "q_out must be 4-byte aligned");
  mf_status st = enqueue_init(h);
  if (st != MF_OK) return st;
  st = enqueue_steps(h, iters);
  if (st != MF_OK) return st;
  if (q_out) {
    const size_t elems = (size_t)h->d.batch * h->d.n_labels * h->d.n_nodes;
    hipError_t e = mf::launch_exp(buf(h, h->cur), q_out, elems, h->stream);
    if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("exp launch: ") + hipGetErrorString(e));
  }
  return MF_OK;
}

mf_status mf_free_energy(mf_handle* h, double* F_host) {
  if (!h) return fail(nullptr, MF_EINVAL, "handle is NULL");
  if (!F_host) return fail(h, MF_EINVAL, "F_host is NULL");
  const mf_desc& d = h->d;
  mf::FreeEnergyArgs a;
  a.unary = d.unary;
  a.state = buf(h, h->cur);
  a.theta = d.theta;
  a.B = d.batch;
  a.L = d.n_labels;
  a.N = d.n_nodes;
  a.H = d.height;
  a.W = d.width;
  a.potts_w = d.potts_w;
  a.partials = (double*)((char*)d.workspace + h->ws.partials);
  a.n_blocks = h->ws.n_blocks;
  double* f_dev = (double*)((char*)d.workspace + h->ws.f_out);
  hipError_t e = mf::launch_grid_free_energy(a, d.graph == MF_GRID4 ? 4 : 8, d.compat, f_dev, h->stream);
  if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("free-energy launch: ") + hipGetErrorString(e));
  e = hipMemcpyAsync(F_host, f_dev, sizeof(double) * d.batch, hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
  return mf_check(h);
}

mf_status mf_check(mf_handle* h) {
  if (!h) return fail(nullptr, MF_EINVAL, "handle is NULL");
  int flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, flags_ptr(h), sizeof(int), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("device error: ") + hipGetErrorString(e));
  if (flag & 1) return fail(h, MF_ENONFINITE, "non-finite unary or initial state");
  return MF_OK;
}

const float* mf_current_state(const mf_handle* h) { return h ? buf(h, h->cur) : nullptr; }

int32_t mf_iteration(const mf_handle* h) { return h ? h->iter : -1; }

int32_t mf_steps_per_launch(const mf_handle* h) { return h ? h->k_launch : -1; }

void mf_destroy(mf_handle* h) { delete h; }

const char* mf_last_error(const mf_handle* h) { return h ? h->err.c_str() : g_err.c_str(); }

mf_status mf_dense_kernel(const float* features, int32_t n, int32_t dim, uint16_t* K_bf16, void* stream) {
  (void)features; (void)n; (void)dim; (void)K_bf16; (void)stream;
  return fail(nullptr, MF_EUNSUPPORTED, "dense kernel builder not available in this build");
}

}  // extern "C"
