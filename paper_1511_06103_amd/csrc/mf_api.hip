// Host library: the C ABI of include/mf.h.  Validation, handle lifetime,
// workspace layout and kernel dispatch.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "mf.h"
#include "mf_internal.h"

struct mf_handle {
  mf_desc d;
  hipStream_t stream = nullptr;
  mf::WorkspaceLayout ws;
  int cur = 0;      // state buffer holding the current iterate
  int iter = 0;     // steps since (re)initialisation
  int k_launch = 1; // steps fused per launch
  bool whole = false;  // the whole grid in one workgroup, every step of a launch in LDS
  bool persist = false;  // one resident workgroup per tile, the halo exchanged each step
  unsigned xtag = 1;     // first unused exchange tag (the exchange area starts zeroed)
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

bool choose_whole_grid(const mf_desc& d);
hipError_t clear_exchange(mf_handle* h);

// Grids the persistent kernel may take (whether the device keeps every tile
// resident is checked when the handle is created): library-chosen launch
// shapes, the fixed step, general Theta with 8 < L <= 32, at most
// kPersistMaxTiles 16 x 16 tiles.
bool persist_possible(const mf_desc& d) {
  if (!is_grid(d.graph) || d.rule != MF_RULE_FIXED || d.steps_per_launch > 0 || choose_whole_grid(d)) return false;
  if (!mf::grid_persist_eligible(d.n_labels, d.compat) || d.height < 1 || d.width < 1) return false;
  const int64_t tiles = (int64_t)d.batch * ((d.width + 15) / 16) * ((d.height + 15) / 16);
  return tiles <= mf::kPersistMaxTiles;
}

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
  if (d.graph == MF_CSR) {
    w.csr_q = off;
    off += align256((size_t)mf::csr_q_bytes(d.precision) * 2 * (size_t)d.batch * (size_t)d.n_nodes *
                    (size_t)mf::csr_label_stride(d.n_labels));
  }
  if (d.graph == MF_DENSE) {
    const size_t B = (size_t)d.batch;
    w.dg = mf::dense_geometry(d.n_nodes, d.batch);
    w.dense_ns = mf::dense_planes(d.precision);
    const size_t Np = (size_t)w.dg.Np;
    w.dq = off;
    off += align256(sizeof(uint16_t) * 2 * B * (size_t)w.dense_ns * 32 * Np);
    w.dk = off;
    off += align256(sizeof(uint16_t) * Np * Np);
    w.ds = off;
    off += align256(sizeof(float) * B * (size_t)w.dg.KS * Np * 32);
    w.dt = off;
    off += align256(sizeof(float) * 2 * B * (size_t)w.dg.NEB * 32);
    w.dqd = off;
    off += align256(sizeof(double) * B * (size_t)d.n_nodes * (size_t)d.n_labels);
  }
  if (d.rule == MF_RULE_MOMENTUM || d.rule == MF_RULE_ADAM) {
    // momentum average (and ADAM second moment) [B][L][N], kept across steps
    const size_t E = (size_t)d.batch * d.n_labels * d.n_nodes;
    w.rule_state = off;
    off += align256(sizeof(float) * E * (d.rule == MF_RULE_ADAM ? 2 : 1));
  }
  if (persist_possible(d)) {
    w.xch = off;
    w.xch_bytes = mf::grid_persist_exchange_bytes(d.batch, d.height, d.width, d.n_labels);
    off += align256(w.xch_bytes);
  }
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
  if (d->rule < MF_RULE_FIXED || d->rule > MF_RULE_SWEEP) return bad("unknown step rule");
  if (d->rule == MF_RULE_MOMENTUM || d->rule == MF_RULE_ADAM) {
    if (!(d->rule_gamma1 >= 0.f && d->rule_gamma1 < 1.f)) return bad("rule_gamma1 must lie in [0, 1)");
  }
  if (d->rule == MF_RULE_ADAM) {
    if (!(d->rule_gamma2 >= 0.f && d->rule_gamma2 < 1.f)) return bad("rule_gamma2 must lie in [0, 1)");
    if (!(d->rule_eps >= 0.f && std::isfinite(d->rule_eps))) return bad("rule_eps must be finite and >= 0");
    if (!(d->rule_v0 >= 0.f && std::isfinite(d->rule_v0))) return bad("rule_v0 must be finite and >= 0");
  }
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
  if (d->n_labels > mf::kSmallLabels && (!is_grid(d->graph) || d->rule != MF_RULE_FIXED)) {
    *msg = "more than 32 labels are implemented for grids with the fixed-step rule";
    return MF_EUNSUPPORTED;
  }
  if (d->rule != MF_RULE_FIXED) {
    if (!is_grid(d->graph)) {
      *msg = "step rules other than MF_RULE_FIXED are implemented for grids";
      return MF_EUNSUPPORTED;
    }
    if (d->precision != MF_P_F32) {
      *msg = "step rules other than MF_RULE_FIXED run with FP32 messages";
      return MF_EUNSUPPORTED;
    }
    if (d->rule == MF_RULE_ADAPTIVE && d->n_labels != 2) return bad("MF_RULE_ADAPTIVE needs n_labels == 2");
  }
  if ((size_t)d->n_labels * (size_t)d->n_nodes >= MF_MAX_LABEL_NODES) {
    *msg = "n_labels * n_nodes must be below MF_MAX_LABEL_NODES per problem";
    return MF_EUNSUPPORTED;
  }
  if (d->graph == MF_CSR &&
      (size_t)d->n_nodes * (size_t)mf::csr_label_stride(d->n_labels) * sizeof(float) >= ((size_t)1 << 32)) {
    *msg = "general graphs: n_nodes * (n_labels rounded up to 4 or 8) * 4 bytes must be below 2^32";
    return MF_EUNSUPPORTED;
  }
  if (d->csr_lanes < 0 || d->csr_lanes > 2) return bad("csr_lanes must be 0, 1 or 2");
  if (d->graph == MF_CSR) {
    if (!d->csr_row_ptr) return bad("csr_row_ptr is NULL");
    if (d->csr_nnz < 0 || d->csr_nnz > INT32_MAX) return bad("csr_nnz out of range");
    if (d->csr_nnz > 0 && !d->csr_col) return bad("csr_col is NULL");
    if (((uintptr_t)d->csr_row_ptr | (uintptr_t)d->csr_col | (uintptr_t)d->csr_w) & 3u)
      return bad("CSR arrays must be 4-byte aligned");
  }
  if (d->graph == MF_DENSE) {
    if (!d->dense_K) return bad("dense_K is NULL");
    if ((uintptr_t)d->dense_K & 15u) return bad("dense_K must be 16-byte aligned");
    if ((uintptr_t)d->cooc & 3u) return bad("cooc must be 4-byte aligned");
    if ((int64_t)d->n_nodes * d->n_nodes > ((int64_t)1 << 40)) return bad("dense N too large");
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

char* ws_at(const mf_handle* h, size_t off) { return (char*)h->d.workspace + off; }

mf::DenseStepArgs dense_args(const mf_handle* h, int from) {
  const mf_desc& d = h->d;
  const mf::WorkspaceLayout& w = h->ws;
  const size_t B = (size_t)d.batch, Np = (size_t)w.dg.Np;
  const size_t plane_elems = B * (size_t)w.dense_ns * 32 * Np;
  const size_t t_elems = B * (size_t)w.dg.NEB * 32;
  const size_t elems = B * d.n_labels * d.n_nodes;
  mf::DenseStepArgs a;
  a.K = d.dense_K;
  a.Kt = (uint16_t*)ws_at(h, w.dk);
  a.unary = d.unary;
  a.state_in = d.state + (size_t)from * elems;
  a.state_out = d.state + (size_t)(from ^ 1) * elems;
  a.q_in = (const uint16_t*)ws_at(h, w.dq) + (size_t)from * plane_elems;
  a.q_out = (uint16_t*)ws_at(h, w.dq) + (size_t)(from ^ 1) * plane_elems;
  a.s_part = (float*)ws_at(h, w.ds);
  a.t_in = (const float*)ws_at(h, w.dt) + (size_t)from * t_elems;
  a.t_out = (float*)ws_at(h, w.dt) + (size_t)(from ^ 1) * t_elems;
  a.theta = d.theta;
  a.cooc = d.cooc;
  a.B = d.batch;
  a.L = d.n_labels;
  a.N = d.n_nodes;
  a.Np = w.dg.Np;
  a.KS = w.dg.KS;
  a.NRB = w.dg.NRB;
  a.NEB = w.dg.NEB;
  a.jchunk = w.dg.jchunk;
  a.alpha = (float)d.alpha;
  a.potts_w = d.potts_w;
  a.inv_n = (float)(1.0 / (double)d.n_nodes);
  return a;
}

void* csr_q(const mf_handle* h, int which) {
  const size_t bytes = (size_t)h->d.batch * h->d.n_nodes * mf::csr_label_stride(h->d.n_labels) *
                       (size_t)mf::csr_q_bytes(h->d.precision);
  return (char*)h->d.workspace + h->ws.csr_q + (size_t)which * bytes;
}

mf::StepArgs grid_args(const mf_handle* h, int from) {
  const mf_desc& d = h->d;
  mf::StepArgs a;
  a.unary = d.unary;
  a.state_in = buf(h, from);
  a.state_out = buf(h, from ^ 1);
  a.theta = d.theta;
  a.B = d.batch;
  a.L = d.n_labels;
  a.N = d.n_nodes;
  a.H = d.height;
  a.W = d.width;
  a.alpha = (float)d.alpha;
  a.potts_w = d.potts_w;
  return a;
}

mf::RuleArgs rule_args(const mf_handle* h, int init, int colour) {
  const mf_desc& d = h->d;
  const size_t E = (size_t)d.batch * d.n_labels * d.n_nodes;
  mf::RuleArgs r;
  float* st = (d.rule == MF_RULE_MOMENTUM || d.rule == MF_RULE_ADAM)
                  ? (float*)((char*)d.workspace + h->ws.rule_state)
                  : nullptr;
  r.mom = st;
  r.sq = (st && d.rule == MF_RULE_ADAM) ? st + E : nullptr;
  r.gamma1 = d.rule_gamma1;
  r.gamma2 = d.rule_gamma2;
  r.eps = d.rule_eps;
  r.v0 = d.rule_v0;
  r.d = (float)(1.0 / d.alpha - 1.0);
  r.init = init;
  r.colour = colour;
  return r;
}

// The flags are cleared when the handle is created and by the mf_check that
// reports them, so a solve does not spend a launch on it.
mf_status enqueue_init(mf_handle* h, bool clear_flags) {
  const mf_desc& d = h->d;
  hipError_t e = hipSuccess;
  if (clear_flags) {
    e = mf::launch_clear_flags(flags_ptr(h), 64, h->stream);
    if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("flag clear: ") + hipGetErrorString(e));
    if (h->persist) {
      // no tag of the exchange area's earlier contents may match a tag of this handle
      e = clear_exchange(h);
      if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("exchange clear: ") + hipGetErrorString(e));
    }
  }
  if (d.graph == MF_CSR) {
    e = mf::launch_csr_check(d.csr_row_ptr, d.csr_col, d.n_nodes, d.csr_nnz, flags_ptr(h), h->stream);
    if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("CSR check launch: ") + hipGetErrorString(e));
  }
  e = mf::launch_init(d.unary, buf(h, 0), d.batch, d.n_labels, d.n_nodes, d.init, flags_ptr(h), h->stream);
  if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("init launch: ") + hipGetErrorString(e));
  if (d.graph == MF_CSR) {
    e = mf::launch_csr_q_from_state(buf(h, 0), csr_q(h, 0), d.batch, d.n_labels, d.n_nodes, d.precision,
                                    h->stream);
    if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("CSR q launch: ") + hipGetErrorString(e));
  }
  if (d.graph == MF_DENSE) {
    // planes and column sums of q^0 go to slot 0: prepare writes the "out" side of from = 1
    mf::DenseStepArgs a = dense_args(h, 1);
    a.state_in = buf(h, 0);
    e = mf::launch_dense_tile_k(a, h->stream);
    if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("dense K tiling launch: ") + hipGetErrorString(e));
    e = mf::launch_dense_prepare(a, h->ws.dense_ns, h->stream);
    if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("dense prepare launch: ") + hipGetErrorString(e));
  }
  if (d.rule == MF_RULE_MOMENTUM || d.rule == MF_RULE_ADAM) {
    // momentum average m(q^0) (and the ADAM second moment v0); log q untouched
    e = mf::launch_grid_rule_step(grid_args(h, 0), rule_args(h, 1, 0), d.graph == MF_GRID4 ? 4 : 8, d.compat,
                                  d.rule, h->stream);
    if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("rule state init: ") + hipGetErrorString(e));
  }
  h->cur = 0;
  h->iter = 0;
  return MF_OK;
}

// A small grid left to the library's choice runs whole in one workgroup:
// up to kWholeMaxSteps steps per launch, all in LDS (a 32 x 32 grid is
// bound by launches otherwise).
bool choose_whole_grid(const mf_desc& d) {
  return is_grid(d.graph) && d.rule == MF_RULE_FIXED && d.steps_per_launch <= 0 &&
         mf::grid_whole_fits(d.n_labels, d.n_nodes);
}

// Steps per launch: small grids (fewer 64 x 4 tiles than four per compute
// unit) are bound by launch and memory latency, so several steps are fused:
// four where Theta S runs on the matrix cores (general Theta, 8 < L <= 32;
// measured fastest on the 256 x 256, L = 21 grid), otherwise three (three
// measured faster than two or four for the VALU kernel).  Larger grids
// stream HBM at one step per launch (16 x 128 x 128 and 2048 x 2048 at
// L = 21 measured fastest at one).
int choose_steps_per_launch(const mf_desc& d) {
  if (!is_grid(d.graph) || d.rule != MF_RULE_FIXED || d.n_labels > mf::kSmallLabels) return 1;
  if (choose_whole_grid(d)) return mf::kWholeMaxSteps;
  const int kmax = mf::grid_max_steps_per_launch(d.n_labels, d.compat, d.precision);
  int k = d.steps_per_launch;
  if (k <= 0) {
    const int64_t tiles = (int64_t)d.batch * ((d.width + mf::kTileX - 1) / mf::kTileX) *
                          ((d.height + mf::kTileY - 1) / mf::kTileY);
    const bool mfma = d.compat == MF_COMPAT_GENERAL && d.n_labels > 8 && d.n_labels <= 32;
    k = tiles >= 4 * 256 ? 1 : (mfma ? 4 : 3);
  }
  return k < kmax ? k : kmax;
}

mf_status enqueue_csr_steps(mf_handle* h, int n) {
  const mf_desc& d = h->d;
  for (; n > 0; --n) {
    mf::CsrStepArgs a;
    a.unary = d.unary;
    a.state_in = buf(h, h->cur);
    a.state_out = buf(h, h->cur ^ 1);
    a.q_in = csr_q(h, h->cur);
    a.q_out = csr_q(h, h->cur ^ 1);
    a.lanes = d.csr_lanes;
    a.row_ptr = d.csr_row_ptr;
    a.col = d.csr_col;
    a.w = d.csr_w;
    a.nnz = d.csr_nnz;
    a.theta = d.theta;
    a.B = d.batch;
    a.L = d.n_labels;
    a.N = d.n_nodes;
    a.alpha = (float)d.alpha;
    a.potts_w = d.potts_w;
    hipError_t e = mf::launch_csr_step(a, d.compat, d.precision, h->stream);
    if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("CSR step launch: ") + hipGetErrorString(e));
    h->cur ^= 1;
    h->iter += 1;
  }
  return MF_OK;
}

mf_status enqueue_dense_steps(mf_handle* h, int n) {
  for (; n > 0; --n) {
    const mf::DenseStepArgs a = dense_args(h, h->cur);
    hipError_t e = mf::launch_dense_step(a, h->ws.dense_ns, h->d.compat, h->stream);
    if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("dense step launch: ") + hipGetErrorString(e));
    h->cur ^= 1;
    h->iter += 1;
  }
  return MF_OK;
}

// Non-fixed step rules: one launch per step; a SWEEP step is one launch per
// colour class, each writing every node (new values for its colour, copies
// for the others) to the other buffer.
mf_status enqueue_rule_steps(mf_handle* h, int n) {
  const mf_desc& d = h->d;
  const int conn = d.graph == MF_GRID4 ? 4 : 8;
  const int launches = d.rule == MF_RULE_SWEEP ? (conn == 4 ? 2 : 4) : 1;
  for (; n > 0; --n) {
    for (int c = 0; c < launches; ++c) {
      hipError_t e = mf::launch_grid_rule_step(grid_args(h, h->cur), rule_args(h, 0, c), conn, d.compat, d.rule,
                                               h->stream);
      if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("rule step launch: ") + hipGetErrorString(e));
      h->cur ^= 1;
    }
    h->iter += 1;
  }
  return MF_OK;
}

mf_status enqueue_steps(mf_handle* h, int n) {
  const mf_desc& d = h->d;
  if (d.graph == MF_CSR) return enqueue_csr_steps(h, n);
  if (d.graph == MF_DENSE) return enqueue_dense_steps(h, n);
  if (d.rule != MF_RULE_FIXED) return enqueue_rule_steps(h, n);
  if (h->persist) {
    const int conn = d.graph == MF_GRID4 ? 4 : 8;
    uint64_t* xch = (uint64_t*)ws_at(h, h->ws.xch);
    while (n > 0) {
      const int ks = n < h->k_launch ? n : h->k_launch;
      hipError_t e = hipSuccess;
      // a launch uses tags xtag .. xtag + ks; past 2^32 the area is cleared and they restart at 1
      if (h->xtag > 0xFFFFFFFFu - (unsigned)ks - 1u) e = clear_exchange(h);
      if (e == hipSuccess)
        e = mf::launch_grid_persist(grid_args(h, h->cur), conn, d.precision, xch, h->xtag, ks, flags_ptr(h), -1,
                                    nullptr, h->stream);
      if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
      h->xtag += (unsigned)ks + 1u;
      h->cur ^= 1;
      h->iter += ks;
      n -= ks;
    }
    return MF_OK;
  }
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
    hipError_t e = h->whole  ? mf::launch_grid_whole(a, conn, d.compat, d.precision, ks, -1, nullptr, nullptr,
                                                      h->stream)
                   : ks == 1 ? mf::launch_grid_step_lanes(a, conn, d.compat, d.precision, h->stream)
                             : mf::launch_grid_multi_step(a, conn, d.compat, d.precision, h->k_launch, ks,
                                                          h->stream);
    if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
    h->cur ^= 1;
    h->iter += ks;
    n -= ks;
  }
  return MF_OK;
}

// Re-initialise, run iters steps and write q (mf_solve after its argument checks).
mf_status solve_impl(mf_handle* h, int iters, float* q_out) {
  if (h->whole && iters > 0) {
    // a small grid held whole by one workgroup: the initialisation, the
    // steps and the write-out of q in as few launches as the step count
    // allows, with the arithmetic of the separate kernels
    const mf_desc& d = h->d;
    const int conn = d.graph == MF_GRID4 ? 4 : 8;
    h->cur = 0;
    h->iter = 0;
    for (int n = iters, first = 1; n > 0; first = 0) {
      const int ks = n < h->k_launch ? n : h->k_launch;
      const mf::StepArgs a = grid_args(h, h->cur);
      hipError_t e = mf::launch_grid_whole(a, conn, d.compat, d.precision, ks, first ? d.init : -1, flags_ptr(h),
                                           n == ks ? q_out : nullptr, h->stream);
      if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
      h->cur ^= 1;
      h->iter += ks;
      n -= ks;
    }
    return MF_OK;
  }
  if (h->persist && iters > 0) {
    // the persistent kernel: the initialisation, the steps and the write-out
    // of q in one launch per kPersistMaxSteps steps, with the arithmetic of
    // the separate kernels
    const mf_desc& d = h->d;
    const int conn = d.graph == MF_GRID4 ? 4 : 8;
    uint64_t* xch = (uint64_t*)ws_at(h, h->ws.xch);
    h->cur = 0;
    h->iter = 0;
    for (int n = iters, first = 1; n > 0; first = 0) {
      const int ks = n < h->k_launch ? n : h->k_launch;
      hipError_t e = hipSuccess;
      if (h->xtag > 0xFFFFFFFFu - (unsigned)ks - 1u) e = clear_exchange(h);
      if (e == hipSuccess)
        e = mf::launch_grid_persist(grid_args(h, h->cur), conn, d.precision, xch, h->xtag, ks, flags_ptr(h),
                                    first ? d.init : -1, n == ks ? q_out : nullptr, h->stream);
      if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
      h->xtag += (unsigned)ks + 1u;
      h->cur ^= 1;
      h->iter += ks;
      n -= ks;
    }
    return MF_OK;
  }
  mf_status st = enqueue_init(h, false);
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

// Enqueue the FP64 free energy of the current state into f_dev[B] (device).
mf_status enqueue_free_energy(mf_handle* h, double* f_dev) {
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
  hipError_t e;
  if (d.graph == MF_CSR) {
    mf::CsrFreeEnergyArgs c;
    c.unary = d.unary;
    c.state = a.state;
    c.theta = d.theta;
    c.row_ptr = d.csr_row_ptr;
    c.col = d.csr_col;
    c.w = d.csr_w;
    c.nnz = d.csr_nnz;
    c.B = d.batch;
    c.L = d.n_labels;
    c.N = d.n_nodes;
    c.potts_w = d.potts_w;
    c.partials = a.partials;
    c.n_blocks = a.n_blocks;
    e = mf::launch_csr_free_energy(c, d.compat, h->stream);
    if (e == hipSuccess) e = mf::launch_reduce_partials(c.partials, c.n_blocks, c.B, f_dev, h->stream);
  } else if (d.graph == MF_DENSE) {
    mf::DenseFreeEnergyArgs c;
    c.K = d.dense_K;
    c.unary = d.unary;
    c.state = a.state;
    c.theta = d.theta;
    c.cooc = d.cooc;
    c.qd = (double*)ws_at(h, h->ws.dqd);
    c.B = d.batch;
    c.L = d.n_labels;
    c.N = d.n_nodes;
    c.potts_w = d.potts_w;
    c.partials = a.partials;
    c.n_blocks = a.n_blocks;
    e = mf::launch_dense_free_energy(c, d.compat, h->stream);
    if (e == hipSuccess) e = mf::launch_reduce_partials(c.partials, c.n_blocks, c.B, f_dev, h->stream);
  } else {
    e = mf::launch_grid_free_energy(a, d.graph == MF_GRID4 ? 4 : 8, d.compat, f_dev, h->stream);
  }
  if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("free-energy launch: ") + hipGetErrorString(e));
  return MF_OK;
}

// Scratch of mf_solve_static: the workspace of a solve, in a device array
// that the library owns (one copy per GPU, held until the process ends), so
// that the call allocates nothing.  In host code the array's name is only a
// stand-in: its device address comes from hipGetSymbolAddress, once per
// device with that device current, and only that address is used.
static __device__ __align__(256) unsigned char scratch[MF_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the current device), or
// nullptr with *err set.
void* scratch_address(hipError_t* err) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess && (dev < 0 || dev >= kMaxDevices)) e = hipErrorInvalidDevice;
  if (e != hipSuccess) {
    *err = e;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// The persistent kernel when the device can keep every tile's workgroup
// resident at once (the occupancy query): no halo recomputation and one
// launch per kPersistMaxSteps steps.
bool choose_persist(const mf_desc& d) {
  if (!persist_possible(d)) return false;
  const int64_t tiles = (int64_t)d.batch * ((d.width + 15) / 16) * ((d.height + 15) / 16);
  return tiles <= mf::grid_persist_capacity(d.n_labels, d.graph == MF_GRID4 ? 4 : 8, d.precision);
}

hipError_t clear_exchange(mf_handle* h) {
  h->xtag = 1;
  return mf::launch_fill_f32((float*)ws_at(h, h->ws.xch), h->ws.xch_bytes / sizeof(float), 0.f, h->stream);
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
  h->whole = choose_whole_grid(*d);
  h->persist = choose_persist(*d);
  if (h->persist) h->k_launch = mf::kPersistMaxSteps;
  const mf_status s2 = enqueue_init(h, true);
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
  return solve_impl(h, iters, q_out);
}

mf_status mf_free_energy(mf_handle* h, double* F_host) {
  if (!h) return fail(nullptr, MF_EINVAL, "handle is NULL");
  if (!F_host) return fail(h, MF_EINVAL, "F_host is NULL");
  double* f_dev = (double*)ws_at(h, h->ws.f_out);
  const mf_status st = enqueue_free_energy(h, f_dev);
  if (st != MF_OK) return st;
  hipError_t e = hipMemcpyAsync(F_host, f_dev, sizeof(double) * h->d.batch, hipMemcpyDeviceToHost, h->stream);
  if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
  return mf_check(h);
}

mf_status mf_marginals(mf_handle* h, float* q_out) {
  if (!h) return fail(nullptr, MF_EINVAL, "handle is NULL");
  if (!q_out || ((uintptr_t)q_out & 3u)) return fail(h, MF_EINVAL, "q_out is NULL or misaligned");
  const size_t elems = (size_t)h->d.batch * h->d.n_labels * h->d.n_nodes;
  hipError_t e = mf::launch_exp(buf(h, h->cur), q_out, elems, h->stream);
  if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("exp launch: ") + hipGetErrorString(e));
  return MF_OK;
}

mf_status mf_check(mf_handle* h) {
  if (!h) return fail(nullptr, MF_EINVAL, "handle is NULL");
  int flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, flags_ptr(h), sizeof(int), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("device error: ") + hipGetErrorString(e));
  if (flag != 0) {
    // reported once: clear for the checks that follow
    e = mf::launch_clear_flags(flags_ptr(h), 64, h->stream);
    if (e != hipSuccess) return fail(h, MF_EDEVICE, std::string("flag clear: ") + hipGetErrorString(e));
  }
  if (flag & 4) return fail(h, MF_EDEVICE, "a halo exchange wait of the persistent grid kernel gave up "
                                          "(its workgroups were not all resident); the iterates are invalid");
  if (flag & 2) return fail(h, MF_EINVAL, "malformed CSR arrays (row_ptr not monotone from 0 to nnz, "
                                         "or a column index out of range)");
  if (flag & 1) return fail(h, MF_ENONFINITE, "non-finite unary or initial state");
  return MF_OK;
}

const float* mf_current_state(const mf_handle* h) { return h ? buf(h, h->cur) : nullptr; }

int32_t mf_iteration(const mf_handle* h) { return h ? h->iter : -1; }

int32_t mf_steps_per_launch(const mf_handle* h) { return h ? h->k_launch : -1; }

void mf_destroy(mf_handle* h) { delete h; }

const char* mf_last_error(const mf_handle* h) { return h ? h->err.c_str() : g_err.c_str(); }

mf_status mf_step_many(mf_handle* const* hs, const int32_t* n_steps, int32_t count) {
  if (count < 0) return fail(nullptr, MF_EINVAL, "count must be >= 0");
  if (count == 0) return MF_OK;
  if (!hs) return fail(nullptr, MF_EINVAL, "hs is NULL");
  if (!n_steps) return fail(nullptr, MF_EINVAL, "n_steps is NULL");
  int rounds = 0;
  for (int i = 0; i < count; ++i) {
    if (!hs[i]) return fail(nullptr, MF_EINVAL, "NULL handle in hs");
    if (n_steps[i] < 0) return fail(hs[i], MF_EINVAL, "n_steps must be >= 0 for every handle");
    if (!is_grid(hs[i]->d.graph)) return fail(hs[i], MF_EUNSUPPORTED, "mf_step_many batches grid problems");
    if (hs[i]->d.rule != MF_RULE_FIXED)
      return fail(hs[i], MF_EUNSUPPORTED, "mf_step_many batches the fixed-step rule");
    if (hs[i]->stream != hs[0]->stream) return fail(hs[i], MF_EINVAL, "handles use different streams");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(hs[i], MF_EINVAL, "handle listed twice");
    rounds = std::max(rounds, (int)n_steps[i]);
  }
  const hipStream_t s = hs[0]->stream;
  std::vector<char> done(count);
  for (int t = 0; t < rounds; ++t) {
    // the handles that take a step in this round
    for (int i = 0; i < count; ++i) done[i] = n_steps[i] <= t;
    for (int g = 0; g < count; ++g) {
      if (done[g]) continue;
      const mf_desc& dg = hs[g]->d;
      if (dg.n_labels > mf::kSmallLabels) {
        // stepped on its own, with the kernel of mf_step at one step per launch
        done[g] = 1;
        mf::StepArgs a = grid_args(hs[g], hs[g]->cur);
        hipError_t e = mf::launch_grid_step_lanes(a, dg.graph == MF_GRID4 ? 4 : 8, dg.compat, dg.precision, s);
        if (e != hipSuccess) return fail(hs[g], MF_EDEVICE, std::string("step launch: ") + hipGetErrorString(e));
        hs[g]->cur ^= 1;
        hs[g]->iter += 1;
        continue;
      }
      // the group of handles sharing the kernel instantiation of hs[g]
      std::vector<mf_handle*> grp;
      for (int i = g; i < count; ++i) {
        const mf_desc& di = hs[i]->d;
        if (!done[i] && di.n_labels == dg.n_labels && di.graph == dg.graph && di.compat == dg.compat &&
            di.precision == dg.precision) {
          grp.push_back(hs[i]);
          done[i] = 1;
        }
      }
      const int conn = dg.graph == MF_GRID4 ? 4 : 8;
      for (size_t c0 = 0; c0 < grp.size(); c0 += mf::kMaxSlots) {
        const size_t c1 = std::min(grp.size(), c0 + (size_t)mf::kMaxSlots);
        mf::ManyArgs m;
        m.count = (int)(c1 - c0);
        m.tile_begin[0] = 0;
        for (size_t k = c0; k < c1; ++k) {
          mf_handle* h = grp[k];
          const mf_desc& d = h->d;
          m.slot[k - c0] = grid_args(h, h->cur);
          m.one_minus_alpha[k - c0] = (float)(1.0 - (double)m.slot[k - c0].alpha);
          m.tile_begin[k - c0 + 1] =
              m.tile_begin[k - c0] + mf::grid_lanes_tiles(d.batch, d.height, d.width, d.n_labels);
        }
        hipError_t e = mf::launch_grid_step_lanes_many(m, dg.n_labels, conn, dg.compat, dg.precision, s);
        if (e != hipSuccess)
          return fail(grp[c0], MF_EDEVICE, std::string("batched step launch: ") + hipGetErrorString(e));
        for (size_t k = c0; k < c1; ++k) {
          grp[k]->cur ^= 1;
          grp[k]->iter += 1;
        }
      }
    }
  }
  return MF_OK;
}

size_t mf_backward_workspace_size(const mf_handle* h, int32_t ckpt_every) {
  if (!h || ckpt_every < 1 || !is_grid(h->d.graph) || h->d.rule != MF_RULE_FIXED || h->d.precision != MF_P_F32 ||
      h->d.n_labels > mf::kSmallLabels)
    return 0;
  const mf_desc& d = h->d;
  const size_t E = (size_t)d.batch * d.n_labels * d.n_nodes;
  const size_t LL = (size_t)d.n_labels * d.n_labels;
  size_t off = 0;
  off += align256(sizeof(float) * E * ((size_t)ckpt_every + 1));   // recomputed states
  off += align256(sizeof(float) * E * 2);                          // gradient ping-pong
  off += align256(sizeof(float) * E);                              // Theta^T m_bar
  off += align256(sizeof(double) * LL * mf::adjoint_theta_parts(d.batch, d.height, d.width));
  off += align256(sizeof(double) * LL);
  off += align256(sizeof(double) * LL * mf::adjoint_theta_stages(d.batch, d.height, d.width));
  return off;
}

mf_status mf_backward(mf_handle* h, const float* ckpt_states, int32_t T, int32_t ckpt_every,
                      const float* grad_logq_T, float* grad_unary, float* grad_theta, void* work,
                      size_t work_bytes) {
  if (!h) return fail(nullptr, MF_EINVAL, "handle is NULL");
  const mf_desc& d = h->d;
  if (!is_grid(d.graph)) return fail(h, MF_EUNSUPPORTED, "the adjoint is implemented for grids");
  if (d.rule != MF_RULE_FIXED) return fail(h, MF_EUNSUPPORTED, "the adjoint is implemented for the fixed-step rule");
  if (d.precision != MF_P_F32)
    return fail(h, MF_EUNSUPPORTED, "the adjoint differentiates the step with FP32 messages only");
  if (d.n_labels > mf::kSmallLabels)
    return fail(h, MF_EUNSUPPORTED, "the adjoint is implemented for at most 32 labels");
  if (T < 0 || ckpt_every < 1) return fail(h, MF_EINVAL, "need T >= 0 and ckpt_every >= 1");
  if (!ckpt_states || !grad_logq_T || !grad_unary || !grad_theta || !work)
    return fail(h, MF_EINVAL, "NULL argument");
  if (((uintptr_t)ckpt_states | (uintptr_t)grad_logq_T | (uintptr_t)grad_unary | (uintptr_t)grad_theta) & 3u)
    return fail(h, MF_EINVAL, "float arrays must be 4-byte aligned");
  if ((uintptr_t)work & 255u) return fail(h, MF_EINVAL, "work must be 256-byte aligned");
  if (work_bytes < mf_backward_workspace_size(h, ckpt_every))
    return fail(h, MF_ENOWORKSPACE, "work smaller than mf_backward_workspace_size");
  const size_t E = (size_t)d.batch * d.n_labels * d.n_nodes;
  const size_t LL = (size_t)d.n_labels * d.n_labels;
  char* w = (char*)work;
  float* R = (float*)w;
  w += align256(sizeof(float) * E * ((size_t)ckpt_every + 1));
  float* G = (float*)w;
  w += align256(sizeof(float) * E * 2);
  float* Sb = (float*)w;
  w += align256(sizeof(float) * E);
  const size_t n_parts = mf::adjoint_theta_parts(d.batch, d.height, d.width);
  double* part = (double*)w;
  w += align256(sizeof(double) * LL * n_parts);
  double* acc = (double*)w;
  w += align256(sizeof(double) * LL);
  double* stage = (double*)w;
  const hipStream_t s = h->stream;
  const int conn = d.graph == MF_GRID4 ? 4 : 8;
  auto dev_fail = [&](hipError_t e, const char* what) {
    return fail(h, MF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e = mf::launch_fill_f32(grad_unary, E, 0.f, s);
  if (e == hipSuccess) e = mf::launch_fill_f64(part, LL * n_parts, s);
  if (e == hipSuccess) e = mf::launch_fill_f64(acc, LL, s);
  if (e == hipSuccess) e = mf::launch_copy_f32(grad_logq_T, G, E, s);
  if (e != hipSuccess) return dev_fail(e, "backward setup");
  int gc = 0;
  const int n_seg = (T + ckpt_every - 1) / ckpt_every;
  for (int seg = n_seg - 1; seg >= 0; --seg) {
    const int t0 = seg * ckpt_every;
    const int len = (t0 + ckpt_every < T ? t0 + ckpt_every : T) - t0;
    e = mf::launch_copy_f32(ckpt_states + (size_t)seg * E, R, E, s);
    if (e != hipSuccess) return dev_fail(e, "checkpoint copy");
    for (int k = 1; k <= len; ++k) {
      mf::StepArgs a;
      a.unary = d.unary;
      a.state_in = R + (size_t)(k - 1) * E;
      a.state_out = R + (size_t)k * E;
      a.theta = d.theta;
      a.B = d.batch;
      a.L = d.n_labels;
      a.N = d.n_nodes;
      a.H = d.height;
      a.W = d.width;
      a.alpha = (float)d.alpha;
      a.potts_w = d.potts_w;
      e = mf::launch_grid_step_lanes(a, conn, d.compat, d.precision, s);
      if (e != hipSuccess) return dev_fail(e, "recompute step");
    }
    for (int k = len - 1; k >= 0; --k) {
      mf::AdjointArgs a;
      a.g_in = G + (size_t)gc * E;
      a.g_out = G + (size_t)(gc ^ 1) * E;
      a.ell_t = R + (size_t)k * E;
      a.ell_t1 = R + (size_t)(k + 1) * E;
      a.u_bar = grad_unary;
      a.s_bar = Sb;
      a.theta = d.theta;
      a.theta_tile = part;
      a.theta_stage = stage;
      a.theta_acc = acc;
      a.B = d.batch;
      a.L = d.n_labels;
      a.N = d.n_nodes;
      a.H = d.height;
      a.W = d.width;
      a.alpha = (float)d.alpha;
      a.potts_w = d.potts_w;
      e = mf::launch_adjoint_step(a, conn, d.compat, s);
      if (e != hipSuccess) return dev_fail(e, "adjoint step");
      gc ^= 1;
    }
  }
  if (d.init == MF_INIT_UNARY) {
    e = mf::launch_adjoint_init(G + (size_t)gc * E, ckpt_states, grad_unary, d.batch, d.n_labels, d.n_nodes, s);
    if (e != hipSuccess) return dev_fail(e, "init adjoint");
  }
  {
    mf::AdjointArgs a;
    a.theta_tile = part;
    a.theta_stage = stage;
    a.theta_acc = acc;
    a.B = d.batch;
    a.L = d.n_labels;
    a.H = d.height;
    a.W = d.width;
    e = mf::launch_adjoint_theta_reduce(a, s);
    if (e != hipSuccess) return dev_fail(e, "theta reduction");
  }
  e = mf::launch_f64_to_f32(acc, grad_theta, LL, s);
  if (e != hipSuccess) return dev_fail(e, "theta gradient");
  return MF_OK;
}

// Workspace of mf_lipschitz: two [L][N] iterates, the scalars, the FP64
// partial sums of one launch.
struct LipLayout {
  size_t a = 0, b = 0, sc = 0, res = 0, part = 0, total = 0;
  int np = 3, blocks = 0;
};

LipLayout lip_layout(const mf_desc& d) {
  LipLayout l;
  const size_t LN = (size_t)d.n_labels * d.n_nodes;
  l.np = d.graph == MF_DENSE ? 3 + mf::kSmallLabels : 3;
  const int hb = mf::lip_blocks(d.graph, d.n_nodes, d.height, d.width);
  const int cb = (d.n_nodes + 255) / 256;
  l.blocks = hb > cb ? hb : cb;
  size_t off = 0;
  l.a = off;
  off += align256(sizeof(float) * LN);
  l.b = off;
  off += align256(sizeof(float) * LN);
  l.sc = off;
  off += align256(sizeof(double) * (2 + mf::kSmallLabels));
  l.res = off;
  off += align256(sizeof(double) * 4);
  l.part = off;
  off += align256(sizeof(double) * (size_t)l.blocks * l.np);
  l.total = off;
  return l;
}

double mf_admissible_alpha(double lipschitz, double margin) {
  if (!(lipschitz > 0.0)) return 1.0;
  if (!(margin >= 1.0)) margin = 1.0;
  return 1.0 / (1.0 + margin * lipschitz);
}

size_t mf_lipschitz_workspace_size(const mf_handle* h) {
  if (!h) return 0;
  return lip_layout(h->d).total;
}

mf_status mf_lipschitz(mf_handle* h, int32_t iters, const float* v0, const float* v1, void* work,
                       size_t work_bytes, double* lambda_max, double* rho) {
  if (!h) return fail(nullptr, MF_EINVAL, "handle is NULL");
  const mf_desc& d = h->d;
  if (iters < 1) return fail(h, MF_EINVAL, "need iters >= 1");
  if (!v0 || !v1 || !work || !lambda_max || !rho) return fail(h, MF_EINVAL, "NULL argument");
  if (((uintptr_t)v0 | (uintptr_t)v1) & 3u) return fail(h, MF_EINVAL, "start vectors must be 4-byte aligned");
  if ((uintptr_t)work & 255u) return fail(h, MF_EINVAL, "work must be 256-byte aligned");
  const LipLayout lay = lip_layout(d);
  if (work_bytes < lay.total) return fail(h, MF_ENOWORKSPACE, "work smaller than mf_lipschitz_workspace_size");
  if (d.n_labels > mf::kSmallLabels)
    return fail(h, MF_EUNSUPPORTED, "the power method is implemented for at most 32 labels");
  if (d.n_labels == 1) {   // the tangent space is {0}
    *lambda_max = 0.0;
    *rho = 0.0;
    return MF_OK;
  }
  char* base = (char*)work;
  float* A = (float*)(base + lay.a);
  float* Bv = (float*)(base + lay.b);
  mf::LipArgs a;
  a.sc = (double*)(base + lay.sc);
  a.res = (double*)(base + lay.res);
  a.part = (double*)(base + lay.part);
  a.np = lay.np;
  a.graph = d.graph;
  a.compat = d.compat;
  a.L = d.n_labels;
  a.N = d.n_nodes;
  a.H = d.height;
  a.W = d.width;
  a.potts_w = d.potts_w;
  a.theta = d.theta;
  a.row_ptr = d.csr_row_ptr;
  a.col = d.csr_col;
  a.csr_w = d.csr_w;
  a.nnz = d.csr_nnz;
  a.K = (const uint16_t*)d.dense_K;
  a.cooc = d.cooc;
  const hipStream_t s = h->stream;
  const int cblocks = (d.n_nodes + 255) / 256;
  const int hblocks = mf::lip_blocks(d.graph, d.n_nodes, d.height, d.width);
  auto dev_fail = [&](hipError_t e, const char* what) {
    return fail(h, MF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  };
  // run 1 on P H P (spectral radius), run 2 on P H P + rho I (lambda_max + rho)
  for (int run = 0; run < 2; ++run) {
    a.v = nullptr;
    a.w = A;
    hipError_t e = mf::launch_lip_center(a, run == 0 ? v0 : v1, s);
    if (e == hipSuccess) e = mf::launch_lip_reduce(a, cblocks, run == 0 ? 0 : 1, s);
    if (e != hipSuccess) return dev_fail(e, "power method start");
    float* cur = A;
    float* nxt = Bv;
    for (int t = 0; t < iters; ++t) {
      a.v = cur;
      a.w = nxt;
      e = mf::launch_lip_hvp(a, s);
      if (e == hipSuccess) e = mf::launch_lip_reduce(a, hblocks, run == 0 ? 2 : 3, s);
      if (e != hipSuccess) return dev_fail(e, "power iteration");
      float* t2 = cur;
      cur = nxt;
      nxt = t2;
    }
  }
  double res[2];
  hipError_t e = hipMemcpyAsync(res, a.res, sizeof(res), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(e, "power method result");
  *rho = res[0];
  *lambda_max = res[1] - res[0];
  return MF_OK;
}

mf_status mf_dense_kernel(const float* features, int32_t n, int32_t dim, uint16_t* K_bf16, void* stream) {
  if (!features || !K_bf16) return fail(nullptr, MF_EINVAL, "features or K is NULL");
  if (n < 1 || dim < 1 || dim > 16) return fail(nullptr, MF_EINVAL, "need n >= 1 and 1 <= dim <= 16");
  if (((uintptr_t)features & 3u) || ((uintptr_t)K_bf16 & 1u)) return fail(nullptr, MF_EINVAL, "misaligned pointer");
  hipError_t e = mf::launch_dense_kernel(features, n, dim, K_bf16, (hipStream_t)stream);
  if (e != hipSuccess) return fail(nullptr, MF_EDEVICE, std::string("dense kernel launch: ") + hipGetErrorString(e));
  return MF_OK;
}

mf_status mf_solve_static(const mf_desc* d, int32_t iters, float* q_out, double* F_out, int32_t* flags_out) {
  if (!d) return fail(nullptr, MF_EINVAL, "descriptor is NULL");
  if (iters < 0) return fail(nullptr, MF_EINVAL, "iters must be >= 0");
  if (((uintptr_t)q_out & 3u) || ((uintptr_t)F_out & 7u) || ((uintptr_t)flags_out & 3u))
    return fail(nullptr, MF_EINVAL, "q_out, F_out or flags_out misaligned");
  if (d->batch < 1 || d->n_nodes < 1 || d->n_labels < 1) return mf_validate(d);
  // the workspace is the static scratch: check the size before any HIP call
  mf_desc dd = *d;
  const size_t need = layout_for(dd).total;
  if (need > MF_STATIC_SCRATCH_BYTES)
    return fail(nullptr, MF_ENOWORKSPACE,
                "problem needs " + std::to_string(need) + " bytes of scratch, above MF_STATIC_SCRATCH_BYTES (" +
                    std::to_string(MF_STATIC_SCRATCH_BYTES) + ")");
  dd.workspace = (void*)(uintptr_t)256;   // placeholder for the host-side checks
  dd.workspace_bytes = MF_STATIC_SCRATCH_BYTES;
  std::string msg;
  const mf_status st = check_desc(&dd, &msg);
  if (st != MF_OK) return fail(nullptr, st, msg);
  hipError_t e = hipSuccess;
  void* ws = scratch_address(&e);
  if (!ws) return fail(nullptr, MF_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
  dd.workspace = ws;
  mf_handle h;   // on the stack: host memory only, nothing allocated on the device
  h.d = dd;
  h.stream = (hipStream_t)dd.stream;
  h.ws = layout_for(dd);
  h.k_launch = choose_steps_per_launch(dd);
  h.whole = choose_whole_grid(dd);
  h.persist = choose_persist(dd);
  if (h.persist) h.k_launch = mf::kPersistMaxSteps;
  // the scratch keeps the previous call's contents: the flags start at zero,
  // and the exchange area holds no tag of this call
  e = mf::launch_clear_flags(flags_ptr(&h), 64, h.stream);
  if (e == hipSuccess && h.persist) e = clear_exchange(&h);
  if (e != hipSuccess) return fail(nullptr, MF_EDEVICE, std::string("flag clear: ") + hipGetErrorString(e));
  mf_status s2 = solve_impl(&h, iters, q_out);
  if (s2 == MF_OK && F_out) s2 = enqueue_free_energy(&h, F_out);
  if (s2 != MF_OK) return fail(nullptr, s2, h.err);
  if (flags_out) {
    e = mf::launch_copy_flags(flags_ptr(&h), flags_out, h.stream);
    if (e != hipSuccess) return fail(nullptr, MF_EDEVICE, std::string("flag copy: ") + hipGetErrorString(e));
  }
  return MF_OK;
}

}  // extern "C"
