// plan.cpp -- the C ABI of libnbs (include/nbs.h): argument checks, the
// compiled channel program, device workspace and the launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/nbs.h"
#include "compiler.hpp"
#include "kernels.hpp"

namespace {

using nbs::CompileOptions;
using nbs::Compiled;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

enum Stage { ST_NEW = 0, ST_BUILT = 1, ST_CONTRACTED = 2 };

}  // namespace

struct nbs_plan_s {
  nbs_geometry geom{};
  int n_ch = 0;
  int prec = 0;
  int device = -1;
  Compiled comp;
  CompileOptions opt;
  std::string err;
  int stage = ST_NEW;
  // device memory
  std::vector<DevBuf> bufs;
  void* Nq = nullptr;
  void* Ft = nullptr;
  int* prog = nullptr;     // all int tables, concatenated
  double* coef = nullptr;  // acc coefficients
  unsigned* maxbits = nullptr;
  int* exps = nullptr;
  double* oscale = nullptr;
  int* chan_nf = nullptr;
  size_t dev_bytes = 0;
  std::map<std::string, size_t> prog_off;  // table name -> offset (ints) into prog
  nbs::NbbArgs nbb{};
  nbs::ContractArgs con{};
};

namespace {

nbs_status fail(nbs_plan p, nbs_status s, const std::string& msg) {
  if (p) p->err = msg;
  return s;
}

bool good_extent(int n) {
  if (n < 2 || n > 128) return false;
  for (int f : {2, 3, 5})
    while (n % f == 0) n /= f;
  return n == 1;
}

int alloc_fail_countdown() {
  const char* e = std::getenv("NBS_TEST_FAIL_ALLOC");
  return e ? std::atoi(e) : 0;
}

nbs_status dev_alloc(nbs_plan p, size_t bytes, void** out, int* countdown) {
  *out = nullptr;
  if (bytes == 0) bytes = 256;
  if (*countdown > 0 && --*countdown == 0)
    return fail(p, NBS_ERR_NOMEM, "injected allocation failure (NBS_TEST_FAIL_ALLOC)");
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) {
    *out = nullptr;
    (void)hipGetLastError();
    return fail(p, NBS_ERR_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  p->bufs.push_back({*out, bytes});
  p->dev_bytes += bytes;
  return NBS_OK;
}

void free_all(nbs_plan p) {
  if (p->device >= 0) {
    (void)hipSetDevice(p->device);
    for (auto& b : p->bufs) (void)hipFree(b.p);
  }
  p->bufs.clear();
}

nbs_status hip_check(nbs_plan p, hipError_t e, const char* what) {
  if (e == hipSuccess) return NBS_OK;
  return fail(p, NBS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Elements of one FFT tile in LDS (two FP64 buffers of this size per
// workgroup): 1024 keeps four workgroups resident per CU.
constexpr int kFftTile = 1024;

constexpr long long kLineMinInner = 16;

int pick_ib(long long inner) {
  for (int ib : {16, 8, 4, 2})
    if (inner % ib == 0) return ib;
  return 1;
}

// Launch the three axis passes of a batched 3-D transform on an array
// [batch][Lz][Ly][Lx][inner0] (inner0 = 3456 for blocks, 1 for F).
nbs_status fft3d(nbs_plan p, int kind_first, int kind_rest, const void* in, void* out, long long batch,
                 const int L[3], long long inner0, int sign, const double* oscale, long long oscale_div,
                 double gscale, hipStream_t st) {
  const long long V = (long long)L[0] * L[1] * L[2];
  for (int ax = 0; ax < 3; ++ax) {
    nbs::FftArgs a{};
    a.in = ax == 0 ? in : out;
    a.out = out;
    a.n = L[ax];
    long long inner = inner0;
    for (int k = 0; k < ax; ++k) inner *= L[k];
    a.inner = inner;
    a.outer = batch * V / ((long long)L[ax] * (inner / inner0));
    a.IB = pick_ib(inner);
    a.OB = std::max(1, kFftTile / (a.IB * a.n));
    a.sign = sign;
    a.gscale = ax == 2 ? gscale : 1.0;
    a.oscale = ax == 2 ? oscale : nullptr;
    a.oscale_div = oscale_div;
    // one line per thread in registers where the length has a kernel and the
    // lines are wide enough apart for adjacent threads to read one run
    const int kind = ax == 0 ? kind_first : kind_rest;
    const bool line = nbs::fft_line_supported(a.n) && inner >= kLineMinInner;
    nbs_status s = hip_check(p, line ? nbs::launch_fft_line(kind, a, st) : nbs::launch_fft_pass(kind, a, st),
                             "fft pass");
    if (s != NBS_OK) return s;
  }
  return NBS_OK;
}

}  // namespace

extern "C" {

const char* nbs_status_string(nbs_status s) {
  switch (s) {
    case NBS_OK: return "ok";
    case NBS_ERR_INVALID: return "invalid argument";
    case NBS_ERR_UNSUPPORTED: return "unsupported";
    case NBS_ERR_NOMEM: return "out of device memory";
    case NBS_ERR_DEVICE: return "device error";
    case NBS_ERR_STATE: return "calls out of order";
  }
  return "unknown status";
}

const char* nbs_last_error(const nbs_plan plan) { return plan ? plan->err.c_str() : "null plan"; }

nbs_status nbs_plan_create(nbs_plan* out, const nbs_geometry* g, int32_t n_geom, const nbs_channel* ch,
                           int32_t n_ch, nbs_precision prec, int32_t device) {
  if (!out) return NBS_ERR_INVALID;
  *out = nullptr;
  if (!g || !ch || n_ch <= 0 || n_geom <= 0) return NBS_ERR_INVALID;
  if (n_geom != 1) return NBS_ERR_UNSUPPORTED;
  if (prec != NBS_FP64 && prec != NBS_FP32_MFMA) return NBS_ERR_INVALID;
  for (int k = 0; k < 3; ++k)
    if (!good_extent(g->L[k])) return NBS_ERR_INVALID;
  if (g->T < 1 || g->t0 < 0 || g->t0 >= g->T || g->t_begin < 0 || g->t_count < 1 ||
      g->t_begin + g->t_count > g->T)
    return NBS_ERR_INVALID;
  const long long V = (long long)g->L[0] * g->L[1] * g->L[2];
  if (V * g->t_count > (1LL << 31) / 32) return NBS_ERR_UNSUPPORTED;

  nbs_plan p = new (std::nothrow) nbs_plan_s;
  if (!p) return NBS_ERR_NOMEM;
  p->geom = *g;
  p->n_ch = n_ch;
  p->prec = prec;
  p->device = device;
  std::vector<nbs::ChannelSpec> specs(n_ch);
  for (int c = 0; c < n_ch; ++c) {
    for (int k = 0; k < 2; ++k) {
      specs[c].sink[k] = ch[c].sink[k];
      specs[c].src[k] = ch[c].src[k];
    }
  }
  p->opt.waves = nbs::contract_waves(prec == NBS_FP64 ? 0 : 1);
  std::string msg = nbs::compile_channels(specs, p->opt, &p->comp);
  if (!msg.empty()) {
    delete p;
    return NBS_ERR_INVALID;
  }
  if (device < 0) {
    if (device != -1) { delete p; return NBS_ERR_INVALID; }
    *out = p;
    return NBS_OK;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) {
    (void)hipGetLastError();
    delete p;
    return NBS_ERR_INVALID;
  }
  if (hipSetDevice(device) != hipSuccess) { delete p; return NBS_ERR_DEVICE; }

  const auto& P = p->comp.prog;
  const int nt = P.n_ops;
  if (nt > nbs::kMaxOps) { delete p; return NBS_ERR_UNSUPPORTED; }
  // diquark flavour pairs and per-operator recipes for the NBB kernel
  nbs::NbbArgs& nb = p->nbb;
  std::map<int, int> dq;
  for (int s = 0; s < nt; ++s) {
    nb.op_nterm[s] = P.op_nterm[s];
    for (int k = 0; k < P.op_nterm[s]; ++k) {
      const int code = P.op_term_trip[3 * s + k];
      const int f1 = code / 9, f2 = (code / 3) % 3, f3 = code % 3;
      const int key = f1 * 3 + f2;
      if (!dq.count(key)) {
        const int id = (int)dq.size();
        if (id >= 4) { delete p; return NBS_ERR_UNSUPPORTED; }
        dq[key] = id;
        nb.dq_f1[id] = f1;
        nb.dq_f2[id] = f2;
      }
      nb.op_dq[s][k] = dq[key];
      nb.op_f3[s][k] = f3;
      nb.op_perm[s][k] = P.op_term_perm[3 * s + k];
      nb.op_w[s][k] = P.op_term_w[3 * s + k];
      nb.flavour_used[f1] = nb.flavour_used[f2] = nb.flavour_used[f3] = 1;
    }
  }
  nb.n_dq = (int)dq.size();
  nb.n_ops = nt;
  nb.V = (int)V;
  nb.t_count = g->t_count;

  const size_t el = prec == NBS_FP64 ? 16 : 8;
  const size_t nq_bytes = (size_t)g->t_count * nt * V * nbs::kBlockEntries * el;
  const size_t ft_bytes = (size_t)n_ch * g->t_count * 16 * V * el;
  // program tables
  std::vector<int> flat;
  auto put = [&](const char* name, const std::vector<int>& v) {
    p->prog_off[name] = flat.size();
    flat.insert(flat.end(), v.begin(), v.end());
    flat.push_back(0);  // keep empty tables addressable
  };
  put("group_op1", P.group_op1); put("group_op2", P.group_op2); put("group_prod", P.group_prod);
  put("group_task", P.group_task); put("group_ch", P.group_ch); put("group_channels", P.group_channels);
  put("ch_contrib", P.ch_contrib); put("contrib_prod", P.contrib_prod); put("prod_desc", P.prod_desc);
  put("task_lanes", P.task_lanes);
  std::vector<int> nf(p->comp.channel_flavour);

  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { (void)hipGetLastError(); free_b = (size_t)-1; }
  const size_t need = nq_bytes + ft_bytes + flat.size() * 4 + P.contrib_coef.size() * 8 + (1 << 20);
  if (need > free_b) {
    delete p;
    return NBS_ERR_NOMEM;
  }
  int countdown = alloc_fail_countdown();
  nbs_status s = NBS_OK;
  void* tmp;
  if ((s = dev_alloc(p, nq_bytes, &p->Nq, &countdown)) != NBS_OK ||
      (s = dev_alloc(p, ft_bytes, &p->Ft, &countdown)) != NBS_OK ||
      (s = dev_alloc(p, flat.size() * 4, &tmp, &countdown)) != NBS_OK) {
    free_all(p);
    delete p;
    return s;
  }
  p->prog = (int*)tmp;
  if ((s = dev_alloc(p, std::max<size_t>(8, P.contrib_coef.size() * 8), &tmp, &countdown)) != NBS_OK) {
    free_all(p); delete p; return s;
  }
  p->coef = (double*)tmp;
  if ((s = dev_alloc(p, 3 * g->t_count * 4, &tmp, &countdown)) != NBS_OK) { free_all(p); delete p; return s; }
  p->maxbits = (unsigned*)tmp;
  if ((s = dev_alloc(p, 3 * g->t_count * 4, &tmp, &countdown)) != NBS_OK) { free_all(p); delete p; return s; }
  p->exps = (int*)tmp;
  if ((s = dev_alloc(p, (size_t)n_ch * g->t_count * 8, &tmp, &countdown)) != NBS_OK) { free_all(p); delete p; return s; }
  p->oscale = (double*)tmp;
  if ((s = dev_alloc(p, nf.size() * 4, &tmp, &countdown)) != NBS_OK) { free_all(p); delete p; return s; }
  p->chan_nf = (int*)tmp;

  hipError_t e = hipMemcpy(p->prog, flat.data(), flat.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && !P.contrib_coef.empty())
    e = hipMemcpy(p->coef, P.contrib_coef.data(), P.contrib_coef.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->chan_nf, nf.data(), nf.size() * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    free_all(p);
    delete p;
    return NBS_ERR_DEVICE;
  }

  nbs::ContractArgs& c = p->con;
  auto T = [&](const char* name) { return (const int*)(p->prog + p->prog_off[name]); };
  c.Nq = p->Nq;
  c.Ft = p->Ft;
  c.V = (int)V;
  c.Lx = g->L[0]; c.Ly = g->L[1]; c.Lz = g->L[2];
  c.t_count = g->t_count;
  c.n_ops = nt;
  c.n_groups = (int)P.group_prod.size() - 1;
  c.n_blocks = (long long)c.n_groups * V * g->t_count;
  if (c.n_blocks + 8 > 0x7fffffffLL) {
    free_all(p);
    delete p;
    return NBS_ERR_UNSUPPORTED;
  }
  c.group_op1 = T("group_op1"); c.group_op2 = T("group_op2"); c.group_prod = T("group_prod");
  c.group_task = T("group_task"); c.group_ch = T("group_ch"); c.group_channels = T("group_channels");
  c.ch_contrib = T("ch_contrib"); c.contrib_prod = T("contrib_prod"); c.prod_desc = T("prod_desc");
  c.task_lanes = T("task_lanes");
  c.contrib_coef = p->coef;
  c.max_gprod = std::max(1, P.max_group_products);
  c.max_gcontrib = std::max(1, P.max_group_contrib);
  c.max_gch = std::max(1, P.max_group_channels);
  c.waves = p->opt.waves;
  if (nbs::contract_lds_bytes(prec, c.max_gprod, c.max_gcontrib, c.max_gch) > 160 * 1024) {
    free_all(p);
    delete p;
    return NBS_ERR_UNSUPPORTED;
  }
  p->nbb.Nq = p->Nq;
  *out = p;
  return NBS_OK;
}

nbs_status nbs_workspace_bytes(const nbs_plan plan, size_t* bytes) {
  if (!plan || !bytes) return NBS_ERR_INVALID;
  *bytes = plan->dev_bytes;
  return NBS_OK;
}

nbs_status nbs_build_blocks(nbs_plan p, const void* const* prop_u, const void* const* prop_d,
                            const void* const* prop_s, void* stream) {
  if (!p) return NBS_ERR_INVALID;
  if (p->device < 0) return fail(p, NBS_ERR_STATE, "host-only plan");
  if (!prop_u || !prop_d || !prop_s || !prop_u[0] || !prop_d[0] || !prop_s[0])
    return fail(p, NBS_ERR_INVALID, "null propagator pointer");
  hipStream_t st = (hipStream_t)stream;
  if (hipSetDevice(p->device) != hipSuccess) return fail(p, NBS_ERR_DEVICE, "hipSetDevice");
  const nbs_geometry& g = p->geom;
  const long long V = (long long)g.L[0] * g.L[1] * g.L[2];
  nbs::NbbArgs a = p->nbb;
  const void* S[3] = {prop_u[0], prop_d[0], prop_s[0]};
  for (int f = 0; f < 3; ++f) a.S[f] = S[f];
  a.scale_exp = nullptr;
  nbs_status s;
  if (p->prec == NBS_FP32_MFMA) {
    if ((s = hip_check(p, nbs::launch_fill_u32(p->maxbits, 0u, 3LL * g.t_count, st), "fill")) != NBS_OK) return s;
    for (int f = 0; f < 3; ++f) {
      if (!a.flavour_used[f]) continue;
      if ((s = hip_check(p, nbs::launch_absmax(S[f], p->maxbits + f * g.t_count, V * 144, g.t_count, st),
                         "absmax")) != NBS_OK)
        return s;
    }
    if ((s = hip_check(p, nbs::launch_scale_exps(p->maxbits, p->exps, 3 * g.t_count, st), "scale")) != NBS_OK)
      return s;
    a.scale_exp = p->exps;
  }
  if ((s = hip_check(p, nbs::launch_nbb(p->prec, a, st), "nbb")) != NBS_OK) return s;
  const int kind = p->prec == NBS_FP64 ? 0 : 1;
  s = fft3d(p, kind, kind, p->Nq, p->Nq, (long long)g.t_count * p->comp.prog.n_ops, g.L, nbs::kBlockEntries,
            -1, nullptr, 1, 1.0, st);
  if (s != NBS_OK) return s;
  p->stage = ST_BUILT;
  return NBS_OK;
}

nbs_status nbs_contract_channels(nbs_plan p, void* stream) {
  if (!p) return NBS_ERR_INVALID;
  if (p->device < 0) return fail(p, NBS_ERR_STATE, "host-only plan");
  if (p->stage < ST_BUILT) return fail(p, NBS_ERR_STATE, "nbs_build_blocks must come first");
  if (hipSetDevice(p->device) != hipSuccess) return fail(p, NBS_ERR_DEVICE, "hipSetDevice");
  nbs_status s = hip_check(p, nbs::launch_contract(p->prec, p->con, (hipStream_t)stream), "contract");
  if (s != NBS_OK) return s;
  p->stage = ST_CONTRACTED;
  return NBS_OK;
}

nbs_status nbs_relative_sum(nbs_plan p, void* const* F_out, void* stream) {
  if (!p) return NBS_ERR_INVALID;
  if (p->device < 0) return fail(p, NBS_ERR_STATE, "host-only plan");
  if (p->stage < ST_CONTRACTED) return fail(p, NBS_ERR_STATE, "nbs_contract_channels must come first");
  if (!F_out || !F_out[0]) return fail(p, NBS_ERR_INVALID, "null output pointer");
  if (hipSetDevice(p->device) != hipSuccess) return fail(p, NBS_ERR_DEVICE, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const nbs_geometry& g = p->geom;
  const double V = (double)g.L[0] * g.L[1] * g.L[2];
  const double* osc = nullptr;
  nbs_status s;
  if (p->prec == NBS_FP32_MFMA) {
    if ((s = hip_check(p, nbs::launch_channel_scale(p->exps, p->chan_nf, p->oscale, p->n_ch, g.t_count, st),
                       "channel scale")) != NBS_OK)
      return s;
    osc = p->oscale;
  }
  const int kfirst = p->prec == NBS_FP64 ? 0 : 2;
  s = fft3d(p, kfirst, 0, p->Ft, F_out[0], (long long)p->n_ch * g.t_count * 16, g.L, 1, +1, osc, 16, 1.0 / V, st);
  if (s != NBS_OK) return s;
  return NBS_OK;
}

nbs_status nbs_plan_destroy(nbs_plan p) {
  if (!p) return NBS_OK;
  if (p->device >= 0) {
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
  }
  free_all(p);
  delete p;
  return NBS_OK;
}

nbs_status nbs_plan_info(const nbs_plan p, nbs_plan_info_t* info) {
  if (!p || !info) return NBS_ERR_INVALID;
  info->n_channels = p->n_ch;
  info->n_types = p->comp.prog.n_ops;
  info->n_diagrams = (int32_t)p->comp.diagrams.size();
  info->n_blocks = p->comp.n_blocks;
  info->n_products = p->comp.n_products;
  info->sum_k = p->comp.sum_k;
  info->n_entries = p->comp.n_entries;
  info->n_terms = p->comp.n_terms;
  info->n_wick_perms = p->comp.n_wick;
  return NBS_OK;
}

nbs_status nbs_plan_diagrams(const nbs_plan p, int32_t ch, nbs_diagram_t* out, int32_t cap, int32_t* n) {
  if (!p || !n || (cap > 0 && !out)) return NBS_ERR_INVALID;
  int cnt = 0;
  for (const auto& d : p->comp.diagrams) {
    if (ch >= 0 && d.channel != ch) continue;
    if (cnt < cap) {
      nbs_diagram_t& o = out[cnt];
      o.channel = d.channel;
      o.src_term = d.src_term;
      o.set1_mask = d.set1_mask;
      o.sign = d.paper_sign;
      o.k = d.k;
      o.labels1 = d.labels1;
      o.open_mask = d.open_mask;
      o.coef = d.coef;
    }
    ++cnt;
  }
  *n = cnt;
  return NBS_OK;
}

nbs_status nbs_plan_table(const nbs_plan p, const char* name, void* buf, int64_t cap, int64_t* n) {
  if (!p || !name || !n || (cap > 0 && !buf)) return NBS_ERR_INVALID;
  const auto& P = p->comp.prog;
  const std::string nm(name);
  const std::vector<double>* dt = nm == "contrib_coef" ? &P.contrib_coef : nm == "op_term_w" ? &P.op_term_w : nullptr;
  if (dt) {
    *n = (int64_t)dt->size();
    if (cap > 0) std::memcpy(buf, dt->data(), sizeof(double) * std::min<int64_t>(cap, *n));
    return NBS_OK;
  }
  const std::map<std::string, const std::vector<int>*> tabs = {
      {"op_code", &P.op_code}, {"op_nterm", &P.op_nterm}, {"op_term_trip", &P.op_term_trip},
      {"op_term_perm", &P.op_term_perm}, {"group_op1", &P.group_op1}, {"group_op2", &P.group_op2},
      {"group_prod", &P.group_prod}, {"group_task", &P.group_task}, {"group_ch", &P.group_ch},
      {"group_channels", &P.group_channels}, {"ch_contrib", &P.ch_contrib}, {"contrib_prod", &P.contrib_prod},
      {"prod_desc", &P.prod_desc}, {"task_lanes", &P.task_lanes}};
  auto it = tabs.find(nm);
  if (it == tabs.end()) return NBS_ERR_INVALID;
  *n = (int64_t)it->second->size();
  if (cap > 0) std::memcpy(buf, it->second->data(), sizeof(int) * std::min<int64_t>(cap, *n));
  return NBS_OK;
}

nbs_status nbs_plan_params(const nbs_plan p, int32_t out[4]) {
  if (!p || !out) return NBS_ERR_INVALID;
  out[0] = nbs::kProdInts;
  out[1] = nbs::kLanesPerTask;
  out[2] = std::max(1, p->comp.prog.max_group_products);
  out[3] = std::max(1, p->comp.prog.max_group_channels);
  return NBS_OK;
}

}  // extern "C"
