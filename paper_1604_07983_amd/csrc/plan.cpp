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

// Per-geometry device workspace.
struct GeomWork {
  nbs_geometry g{};
  long long V = 0;
  void* Nq = nullptr;          // operator blocks (nbs::BlockLayout), then N~(q) in place
  void* Ft = nullptr;          // [n_ch][t_count][16][V] F~_c(q)
  unsigned* maxbits = nullptr; // precision form: [3][t_count] max |Re|, |Im| as float bits
  int* exps = nullptr;         // precision form: [3][t_count] power-of-two exponents
  double* oscale = nullptr;    // precision form: [n_ch][t_count] un-scaling factors
};

// Launch-shape choices (set by nbs_plan_autotune, else the defaults).
struct Tuning {
  int fft_tile = 1024;  // elements of an LDS tile of k_fft_pass (FP64 pairs)
  int fft_line = 1;     // 1: register line kernel where the length has one
  int fft_plane = 1;    // 1: fused x-y pass for square planes of the block transforms
  int fft_cube = 1;     // 1: one pass for all three axes of cubic block transforms
  int split = 1;        // 1: compiler may split the walked index of a product over lanes
  int waves = 8;        // wavefronts per contraction workgroup
  int mfma = 0;         // precision form: 4 x 4-row products on matrix cores
  // contraction workgroups per (slice, momentum): 0 one walking every
  // sink-operator group, 1 one per run of groups in which one operator
  // block stays, 2 one per group
  int gchunk = 0;
  // contraction engine: 0 lane teams on the vector units, 1 segments on the
  // matrix cores; wavefronts per workgroup of the matrix-core engine
  int engine = 1;
  int seg_waves = 16;
  // matrix-core engine: 1 resident workgroups claiming work items from
  // counters, 0 one workgroup per item
  int persist = 0;
};

}  // namespace

struct nbs_plan_s {
  std::vector<GeomWork> gw;
  int n_ch = 0;
  int prec = 0;
  int device = -1;
  std::vector<nbs::ChannelSpec> specs;
  Compiled comp;
  CompileOptions opt;
  Tuning tune;
  std::string err;
  int stage = ST_NEW;
  // device memory
  std::vector<DevBuf> bufs;
  int* prog = nullptr;     // all int tables of the compiled program, concatenated
  double* coef = nullptr;  // channel coefficients
  double* coef_iso = nullptr;  // the same with the isospin alias factors
  bool iso = false;            // last build used the isospin-symmetric limit (prop_d == prop_u)
  int* chan_nf = nullptr;  // [n_ch][3] quark counts
  nbs::ContractGeom* geo = nullptr;
  unsigned* nonfinite = nullptr;  // set by the block kernel on NaN / infinite propagator entries
  unsigned* queue = nullptr;      // eight work-item counters of the persistent contraction
  long long n_qt = 0;  // (slice, momentum) pairs over all geometries
  size_t dev_bytes = 0;
  std::map<std::string, size_t> prog_off;  // table name -> offset (ints) into prog
  nbs::NbbArgs nbb{};                      // geometry-independent part
  nbs::ContractArgs con{};
  nbs::BlockLayout lay{};                  // operator blocks in HBM
  long long lay_entries = 0;               // entries per site over all operators
  // captured launch sequence (nbs_run_graph)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> graph_key;
  // plans without device allocation: every buffer is carved from a caller
  // workspace (arena), tables are uploaded on `upload` and waited for
  char* arena = nullptr;
  size_t arena_size = 0, arena_used = 0;
  hipStream_t upload = nullptr;
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
  if (p->arena) {
    const size_t at = (p->arena_used + 255) & ~(size_t)255;
    if (at + bytes > p->arena_size)
      return fail(p, NBS_ERR_UNSUPPORTED,
                  "the problem needs more device memory than the " + std::to_string(p->arena_size >> 20) +
                      " MiB static workspace holds");
    *out = p->arena + at;
    p->arena_used = at + bytes;
    p->dev_bytes = p->arena_used;
    return NBS_OK;
  }
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

void dev_free(nbs_plan p, void* ptr) {
  if (p->arena) return;  // the caller's workspace is not freed piecewise
  for (size_t i = 0; i < p->bufs.size(); ++i)
    if (p->bufs[i].p == ptr) {
      (void)hipFree(ptr);
      p->dev_bytes -= p->bufs[i].bytes;
      p->bufs.erase(p->bufs.begin() + i);
      return;
    }
}

void drop_graph(nbs_plan p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  p->graph_key.clear();
}

void free_all(nbs_plan p) {
  if (p->arena) {
    p->bufs.clear();
    return;
  }
  if (p->device >= 0) {
    (void)hipSetDevice(p->device);
    drop_graph(p);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    p->cap_stream = nullptr;
    for (auto& b : p->bufs) (void)hipFree(b.p);
  }
  p->bufs.clear();
}

// Host-to-device copy of a table: synchronous for allocating plans; for
// workspace plans ordered on their stream and waited for (the host buffer
// is freed after the call).
hipError_t upload(nbs_plan p, void* dst, const void* src, size_t bytes) {
  if (!p->arena) return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
  hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, p->upload);
  if (e == hipSuccess) e = hipStreamSynchronize(p->upload);
  return e;
}

nbs_status hip_check(nbs_plan p, hipError_t e, const char* what) {
  if (e == hipSuccess) return NBS_OK;
  return fail(p, NBS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr long long kLineMinInner = 16;

int pick_ib(long long inner) {
  for (int ib : {16, 8, 4, 2})
    if (inner % ib == 0) return ib;
  return 1;
}

// Launch the three axis passes of a batched 3-D transform on an array
// [batch][Lz][Ly][Lx][inner0] (inner0 = an operator's block entries, 1 for F).
nbs_status fft3d(nbs_plan p, int kind_first, int kind_rest, const void* in, void* out, long long batch,
                 const int L[3], long long inner0, int sign, const double* oscale, long long oscale_div,
                 double gscale, hipStream_t st) {
  const long long V = (long long)L[0] * L[1] * L[2];
  int ax0 = 0;
  // contiguous cubic fields of the inverse transform: all three axes in one pass
  if (p->tune.fft_cube && sign > 0 && inner0 == 1 && L[0] == L[1] && L[1] == L[2] && kind_rest == 0 &&
      nbs::fft_cube_inv_supported(L[0], kind_first)) {
    nbs::FftArgs a{};
    a.in = in;
    a.out = out;
    a.outer = batch;
    a.inner = 1;
    a.n = L[0];
    a.sign = sign;
    a.gscale = gscale;
    a.oscale = oscale;
    a.oscale_div = oscale_div;
    return hip_check(p, nbs::launch_fft_cube_inv(kind_first, a, st), "fft cube inverse");
  }
  // cubic lattices of a forward block transform: all three axes in one pass
  const int cib = p->tune.fft_cube && L[0] == L[1] && L[1] == L[2] && sign < 0 && oscale == nullptr &&
                          gscale == 1.0 && kind_first == kind_rest
                      ? nbs::fft_cube_fields(L[0], inner0, kind_first)
                      : 0;
  if (cib > 0) {
    nbs::FftPlaneArgs ca{};
    ca.in = in;
    ca.out = out;
    ca.planes = batch;
    ca.inner = inner0;
    ca.IB = cib;
    return hip_check(p, nbs::launch_fft_cube(kind_first, L[0], ca, st), "fft cube");
  }
  // square x-y planes of a forward block transform: both axes in one pass
  const int pib = p->tune.fft_plane && L[0] == L[1] && sign < 0 && oscale == nullptr && gscale == 1.0 &&
                          kind_first == kind_rest
                      ? nbs::fft_plane_fields(L[0], inner0, kind_first)
                      : 0;
  if (pib > 0) {
    nbs::FftPlaneArgs pa{};
    pa.in = in;
    pa.out = out;
    pa.planes = batch * L[2];
    pa.inner = inner0;
    pa.IB = pib;
    nbs_status s = hip_check(p, nbs::launch_fft_plane(kind_first, L[0], pa, st), "fft plane");
    if (s != NBS_OK) return s;
    ax0 = 2;
  }
  for (int ax = ax0; ax < 3; ++ax) {
    nbs::FftArgs a{};
    a.in = ax == 0 ? in : out;  // after the fused x-y pass the data is in out
    a.out = out;
    a.n = L[ax];
    long long inner = inner0;
    for (int k = 0; k < ax; ++k) inner *= L[k];
    a.inner = inner;
    a.outer = batch * V / ((long long)L[ax] * (inner / inner0));
    a.IB = pick_ib(inner);
    a.OB = std::max(1, p->tune.fft_tile / (a.IB * a.n));
    // two FP64 tiles and the twiddles must fit the 160 KB of LDS
    while (a.OB > 1 && 16.0 * (a.n + 2.0 * a.OB * a.IB * (a.n + 1)) > 160.0 * 1024) a.OB /= 2;
    a.sign = sign;
    a.gscale = ax == 2 ? gscale : 1.0;
    a.oscale = ax == 2 ? oscale : nullptr;
    a.oscale_div = oscale_div;
    // one line per thread in registers where the length has a kernel and the
    // lines are wide enough apart for adjacent threads to read one run
    const int kind = ax == 0 ? kind_first : kind_rest;
    const bool line = p->tune.fft_line && nbs::fft_line_supported(a.n, kind) && inner >= kLineMinInner;
    nbs_status s = hip_check(p, line ? nbs::launch_fft_line(kind, a, st) : nbs::launch_fft_pass(kind, a, st),
                             "fft pass");
    if (s != NBS_OK) return s;
  }
  return NBS_OK;
}

// Boundaries of the ranges of groups one contraction workgroup walks (mode
// as Tuning::gchunk): [0, n), the runs in which one operator block stays,
// or single groups.
std::vector<int> group_chunks(const std::vector<int>& op1, const std::vector<int>& op2, int mode) {
  const int n = (int)op1.size();
  std::vector<int> b{0};
  for (int g = 1; g < n; ++g)
    if (mode == 2 || (mode == 1 && op1[g] != op1[g - 1] && op2[g] != op2[g - 1])) b.push_back(g);
  b.push_back(n);
  if (n == 0) b = {0, 0};
  return b;
}

// Compile the channel table with the plan's options and (device plans)
// upload its tables, replacing earlier ones.
nbs_status compile_and_upload(nbs_plan p) {
  p->opt.waves = p->tune.waves;
  p->opt.split = p->tune.split != 0;
  p->opt.mfma = p->prec == NBS_FP32_MFMA && p->tune.mfma != 0;
  p->opt.seg_waves = p->tune.seg_waves;
  p->opt.fp32 = p->prec == NBS_FP32_MFMA;
  p->opt.max_group_slots = 128;
  Compiled comp;
  std::string msg = nbs::compile_channels(p->specs, p->opt, &comp);
  if (!msg.empty()) return fail(p, NBS_ERR_INVALID, msg);
  p->comp = std::move(comp);
  if (p->device < 0) return NBS_OK;
  const auto& P = p->comp.prog;
  std::vector<int> flat;
  std::map<std::string, size_t> off;
  auto put = [&](const char* name, const std::vector<int>& v) {
    off[name] = flat.size();
    flat.insert(flat.end(), v.begin(), v.end());
    flat.push_back(0);  // keep empty tables addressable
  };
  put("group_op1", P.group_op1); put("group_op2", P.group_op2); put("group_prod", P.group_prod);
  put("group_task", P.group_task); put("group_ch", P.group_ch); put("group_channels", P.group_channels);
  put("ch_contrib", P.ch_contrib); put("contrib_prod", P.contrib_prod); put("prod_desc", P.prod_desc);
  put("task_lanes", P.task_lanes);
  put("group_op1_iso", P.group_op1_iso); put("group_op2_iso", P.group_op2_iso);
  put("seg_task", P.seg_task); put("group_stask", P.group_stask); put("prod_ext", P.prod_ext);
  put("contrib_ext", P.contrib_ext);
  const std::vector<int> gchunk = group_chunks(P.group_op1, P.group_op2, p->tune.gchunk);
  put("gchunk", gchunk);
  int countdown = 0;
  void* prog = nullptr;
  void* coef = nullptr;
  nbs_status s = dev_alloc(p, flat.size() * 4, &prog, &countdown);
  if (s != NBS_OK) return s;
  void* coef_iso = nullptr;
  if ((s = dev_alloc(p, std::max<size_t>(8, P.contrib_coef.size() * 8), &coef, &countdown)) != NBS_OK) {
    dev_free(p, prog);
    return s;
  }
  if ((s = dev_alloc(p, std::max<size_t>(8, P.contrib_coef_iso.size() * 8), &coef_iso, &countdown)) != NBS_OK) {
    dev_free(p, prog);
    dev_free(p, coef);
    return s;
  }
  hipError_t e = upload(p, prog, flat.data(), flat.size() * 4);
  if (e == hipSuccess && !P.contrib_coef.empty()) e = upload(p, coef, P.contrib_coef.data(), P.contrib_coef.size() * 8);
  if (e == hipSuccess && !P.contrib_coef_iso.empty())
    e = upload(p, coef_iso, P.contrib_coef_iso.data(), P.contrib_coef_iso.size() * 8);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    dev_free(p, prog);
    dev_free(p, coef);
    dev_free(p, coef_iso);
    return fail(p, NBS_ERR_DEVICE, "table upload");
  }
  if (p->prog) dev_free(p, p->prog);
  if (p->coef) dev_free(p, p->coef);
  if (p->coef_iso) dev_free(p, p->coef_iso);
  p->prog = (int*)prog;
  p->coef = (double*)coef;
  p->coef_iso = (double*)coef_iso;
  p->prog_off = off;
  nbs::ContractArgs& c = p->con;
  auto T = [&](const char* name) { return (const int*)(p->prog + p->prog_off[name]); };
  c.n_ops = P.n_ops;
  c.n_groups = (int)P.group_prod.size() - 1;
  c.group_op1 = T("group_op1"); c.group_op2 = T("group_op2"); c.group_prod = T("group_prod");
  c.group_task = T("group_task"); c.group_ch = T("group_ch"); c.group_channels = T("group_channels");
  c.ch_contrib = T("ch_contrib"); c.contrib_prod = T("contrib_prod"); c.prod_desc = T("prod_desc");
  c.task_lanes = T("task_lanes");
  c.gchunk = T("gchunk");
  c.n_gchunk = (int)gchunk.size() - 1;
  c.n_blocks = p->n_qt * c.n_gchunk;
  c.contrib_coef = p->coef;
  c.max_gprod = std::max(1, P.max_group_products);
  c.max_gcontrib = std::max(1, P.max_group_contrib);
  c.max_gch = std::max(1, P.max_group_channels);
  c.max_gtask = std::max(1, P.max_group_tasks);
  c.engine = p->tune.engine;
  c.seg_task = T("seg_task");
  c.group_stask = T("group_stask");
  c.prod_ext = T("prod_ext");
  c.contrib_ext = T("contrib_ext");
  c.max_gslots = std::max(1, P.max_group_slots);
  c.max_gstask = std::max(1, P.max_group_stasks);
  c.waves = c.engine == 1 ? p->tune.seg_waves : p->tune.waves;
  c.lay = p->lay;
  c.persistent = c.engine == 1 ? p->tune.persist : 0;
  c.queue = p->queue;
  // result slots spaced kSegRStride apart where the LDS allows it
  c.rstride = nbs::kSegRStride;
  if (nbs::contract_seg_lds_bytes(p->prec, c.max_gslots, c.max_gcontrib, c.max_gch, c.max_gstask, c.rstride) >
      160 * 1024)
    c.rstride = 16;
  const size_t lds = c.engine == 1 ? nbs::contract_seg_lds_bytes(p->prec, c.max_gslots, c.max_gcontrib, c.max_gch,
                                                                 c.max_gstask, c.rstride)
                                   : nbs::contract_lds_bytes(p->prec, c.max_gprod, c.max_gcontrib, c.max_gch, c.max_gtask);
  if (lds > 160 * 1024) return fail(p, NBS_ERR_UNSUPPORTED, "a channel group needs more LDS than a CU has");
  return hip_check(p, nbs::prepare_kernels(p->prec, c.waves, lds, c.engine), "kernel attributes");
}

// ---- the three stages, enqueued on a stream --------------------------------

// The isospin-symmetric limit holds when every geometry's d propagator is
// the u propagator (the same memory).
bool isospin_limit(nbs_plan p, const void* const* pu, const void* const* pd) {
  if (p->comp.prog.n_canon >= p->comp.prog.n_ops) return false;
  for (size_t i = 0; i < p->gw.size(); ++i)
    if (pu[i] != pd[i]) return false;
  return true;
}

// Forward transform of the first n_build operators' blocks of one geometry,
// operator by operator (each [t][site][ne] with its own field count).
nbs_status transform_blocks(nbs_plan p, GeomWork& w, int n_build, hipStream_t st) {
  const int kind = p->prec == NBS_FP64 ? 0 : 1;
  const size_t el = p->prec == NBS_FP64 ? 16 : 8;
  for (int op = 0; op < n_build; ++op) {
    char* base = (char*)w.Nq + (size_t)p->lay.cum[op] * w.g.t_count * w.V * el;
    const nbs_status s =
        fft3d(p, kind, kind, base, base, (long long)w.g.t_count, w.g.L, p->lay.ne[op], -1, nullptr, 1, 1.0, st);
    if (s != NBS_OK) return s;
  }
  return NBS_OK;
}

nbs_status enqueue_build(nbs_plan p, const void* const* pu, const void* const* pd, const void* const* ps,
                         hipStream_t st) {
  nbs_status s;
  // in the isospin-symmetric limit only the canonical operator blocks (the
  // first n_canon slots) are built and transformed (Sec. 4(i))
  p->iso = isospin_limit(p, pu, pd);
  const int n_build = p->iso ? p->comp.prog.n_canon : p->comp.prog.n_ops;
  // the non-finite input flag of this block build (a fill kernel, not a memset,
  // so that the sequence can be captured into a graph)
  if ((s = hip_check(p, nbs::launch_fill_u32(p->nonfinite, 0u, 1, st), "fill")) != NBS_OK) return s;
  for (size_t i = 0; i < p->gw.size(); ++i) {
    GeomWork& w = p->gw[i];
    const nbs_geometry& g = w.g;
    nbs::NbbArgs a = p->nbb;
    const void* S[3] = {pu[i], pd[i], ps[i]};
    for (int f = 0; f < 3; ++f) a.S[f] = S[f];
    a.Nq = w.Nq;
    a.V = (int)w.V;
    a.t_count = g.t_count;
    a.n_ops = n_build;
    a.scale_exp = nullptr;
    a.nonfinite = p->nonfinite;
    if (p->prec == NBS_FP32_MFMA) {
      if ((s = hip_check(p, nbs::launch_fill_u32(w.maxbits, 0u, 3LL * g.t_count, st), "fill")) != NBS_OK) return s;
      for (int f = 0; f < 3; ++f) {
        if (!a.flavour_used[f]) continue;
        if ((s = hip_check(p, nbs::launch_absmax(S[f], w.maxbits + f * g.t_count, w.V * 144, g.t_count, st),
                           "absmax")) != NBS_OK)
          return s;
      }
      if ((s = hip_check(p, nbs::launch_scale_exps(w.maxbits, w.exps, 3 * g.t_count, st), "scale")) != NBS_OK)
        return s;
      a.scale_exp = w.exps;
    }
    if ((s = hip_check(p, nbs::launch_nbb(p->prec, a, st), "nbb")) != NBS_OK) return s;
    if ((s = transform_blocks(p, w, n_build, st)) != NBS_OK) return s;
  }
  return NBS_OK;
}

nbs_status enqueue_contract(nbs_plan p, hipStream_t st) {
  nbs::ContractArgs a = p->con;
  if (a.persistent) {
    // the work-item counters start at zero (a fill kernel, not a memset,
    // so that the sequence can be captured into a graph)
    nbs_status s = hip_check(p, nbs::launch_fill_u32(p->queue, 0u, 8, st), "fill");
    if (s != NBS_OK) return s;
    a.queue = p->queue;
  }
  if (p->iso) {
    a.group_op1 = (const int*)(p->prog + p->prog_off["group_op1_iso"]);
    a.group_op2 = (const int*)(p->prog + p->prog_off["group_op2_iso"]);
    a.contrib_coef = p->coef_iso;
  }
  return hip_check(p, nbs::launch_contract(p->prec, a, st), "contract");
}

nbs_status enqueue_relsum(nbs_plan p, void* const* F_out, hipStream_t st) {
  nbs_status s;
  for (size_t i = 0; i < p->gw.size(); ++i) {
    GeomWork& w = p->gw[i];
    const nbs_geometry& g = w.g;
    const double* osc = nullptr;
    if (p->prec == NBS_FP32_MFMA) {
      if ((s = hip_check(p, nbs::launch_channel_scale(w.exps, p->chan_nf, w.oscale, p->n_ch, g.t_count, st),
                         "channel scale")) != NBS_OK)
        return s;
      osc = w.oscale;
    }
    const int kfirst = p->prec == NBS_FP64 ? 0 : 2;
    s = fft3d(p, kfirst, 0, w.Ft, F_out[i], (long long)p->n_ch * g.t_count * 16, g.L, 1, +1, osc, 16,
              1.0 / (double)w.V, st);
    if (s != NBS_OK) return s;
  }
  return NBS_OK;
}

bool ptrs_ok(const void* const* a, size_t n) {
  if (!a) return false;
  for (size_t i = 0; i < n; ++i)
    if (!a[i]) return false;
  return true;
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

}  // extern "C"

namespace nbs {

namespace {
thread_local std::string t_create_err;  // why the last create_plan of this thread failed
}

const char* create_error() { return t_create_err.c_str(); }

nbs_status create_plan(nbs_plan* out, const nbs_geometry* g, int32_t n_geom, const nbs_channel* ch, int32_t n_ch,
                       nbs_precision prec, int32_t device, void* arena, size_t arena_size, hipStream_t upload_stream) {
  t_create_err.clear();
  if (!out) return NBS_ERR_INVALID;
  *out = nullptr;
  if (!g || !ch || n_ch <= 0 || n_geom <= 0) return NBS_ERR_INVALID;
  if (n_geom > nbs::kMaxGeom) return NBS_ERR_UNSUPPORTED;
  if (prec != NBS_FP64 && prec != NBS_FP32_MFMA) return NBS_ERR_INVALID;
  for (int i = 0; i < n_geom; ++i) {
    for (int k = 0; k < 3; ++k)
      if (!good_extent(g[i].L[k])) return NBS_ERR_INVALID;
    if (g[i].T < 1 || g[i].t0 < 0 || g[i].t0 >= g[i].T || g[i].t_begin < 0 || g[i].t_count < 1 ||
        g[i].t_begin + g[i].t_count > g[i].T)
      return NBS_ERR_INVALID;
    const long long V = (long long)g[i].L[0] * g[i].L[1] * g[i].L[2];
    if (V * g[i].t_count > (1LL << 31) / 32) return NBS_ERR_UNSUPPORTED;
  }

  nbs_plan p = new (std::nothrow) nbs_plan_s;
  if (!p) return NBS_ERR_NOMEM;
  if (arena) {
    if (device < 0) {
      delete p;
      return NBS_ERR_INVALID;
    }
    p->arena = (char*)arena;
    p->arena_size = arena_size;
    p->upload = upload_stream;
  }
  p->n_ch = n_ch;
  p->prec = prec;
  p->device = device;
  p->gw.resize(n_geom);
  for (int i = 0; i < n_geom; ++i) {
    p->gw[i].g = g[i];
    p->gw[i].V = (long long)g[i].L[0] * g[i].L[1] * g[i].L[2];
  }
  p->specs.resize(n_ch);
  for (int c = 0; c < n_ch; ++c)
    for (int k = 0; k < 2; ++k) {
      p->specs[c].sink[k] = ch[c].sink[k];
      p->specs[c].src[k] = ch[c].src[k];
    }
  p->tune.waves = nbs::contract_waves(prec == NBS_FP64 ? 0 : 1);
  // matrix-core engine: 512-thread workgroups (measured faster than 1024 in
  // both forms; in the precision form two of them share a CU)
  p->tune.seg_waves = 8;
  // the fused x-y pass pays off for FP64 storage (128-byte runs in 64 KB
  // tiles at 16^3); for complex64 the separate passes measured faster at
  // 32^3 and 40^3.  8^3 and 16^3 cubes take the one-pass transform in both
  // forms (measured faster than either at 16^3).
  p->tune.fft_plane = prec == NBS_FP64 ? 1 : 0;
  p->tune.fft_cube = 1;
  // matrix-core products are an autotuner candidate: measured slower than
  // the vector loops for these 4 x 4 products (a quad walks a product's
  // shared indices one step at a time, four times the steps of a lane team)
  p->tune.mfma = 0;
  // workgroups that walk every group measured fastest in both forms
  p->tune.gchunk = 0;
  if (device < -1) { delete p; return NBS_ERR_INVALID; }
  if (device >= 0) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) {
      (void)hipGetLastError();
      delete p;
      return NBS_ERR_INVALID;
    }
    if (hipSetDevice(device) != hipSuccess) { delete p; return NBS_ERR_DEVICE; }
  }
  {
    // compile only (device tables come after the workspace)
    const int dev = p->device;
    p->device = -1;
    const nbs_status s = compile_and_upload(p);
    p->device = dev;
    if (s != NBS_OK) {
      t_create_err = p->err;
      delete p;
      return s;
    }
  }
  if (device < 0) {
    *out = p;
    return NBS_OK;
  }

  const auto& P = p->comp.prog;
  const int nt = P.n_ops;
  if (nt > nbs::kMaxOps) { delete p; return NBS_ERR_UNSUPPORTED; }
  // diquark flavour pairs and per-operator recipes for the NBB kernel
  // block layout: operators with a stored antisymmetrised pair packed
  {
    int cum = 0;
    for (int s = 0; s < nt; ++s) {
      p->lay.pair[s] = P.op_pair[s];
      p->lay.ne[s] = P.op_pair[s] >= 0 ? nbs::kPackedEntries : nbs::kBlockEntries;
      p->lay.cum[s] = cum;
      cum += p->lay.ne[s];
    }
    p->lay_entries = cum;
  }
  nbs::NbbArgs& nb = p->nbb;
  nb.lay = p->lay;
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

  // workspace of every geometry
  const size_t el = prec == NBS_FP64 ? 16 : 8;
  size_t need = (1 << 22);
  long long n_qt = 0;
  for (auto& w : p->gw) {
    need += (size_t)w.g.t_count * p->lay_entries * w.V * el + (size_t)n_ch * w.g.t_count * 16 * w.V * el;
    n_qt += w.V * w.g.t_count;
  }
  if (!p->arena) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { (void)hipGetLastError(); free_b = (size_t)-1; }
    if (need > free_b) {
      delete p;
      return NBS_ERR_NOMEM;
    }
  }
  int countdown = p->arena ? 0 : alloc_fail_countdown();
  nbs_status s = NBS_OK;
  void* tmp = nullptr;
  auto bail = [&](nbs_status st) {
    t_create_err = p->err;
    free_all(p);
    delete p;
    return st;
  };
  for (auto& w : p->gw) {
    const int tc = w.g.t_count;
    if ((s = dev_alloc(p, (size_t)tc * p->lay_entries * w.V * el, &w.Nq, &countdown)) != NBS_OK ||
        (s = dev_alloc(p, (size_t)n_ch * tc * 16 * w.V * el, &w.Ft, &countdown)) != NBS_OK)
      return bail(s);
    if ((s = dev_alloc(p, 3 * tc * 4, &tmp, &countdown)) != NBS_OK) return bail(s);
    w.maxbits = (unsigned*)tmp;
    if ((s = dev_alloc(p, 3 * tc * 4, &tmp, &countdown)) != NBS_OK) return bail(s);
    w.exps = (int*)tmp;
    if ((s = dev_alloc(p, (size_t)n_ch * tc * 8, &tmp, &countdown)) != NBS_OK) return bail(s);
    w.oscale = (double*)tmp;
  }
  const std::vector<int>& nf = p->comp.channel_flavour;
  if ((s = dev_alloc(p, nf.size() * 4, &tmp, &countdown)) != NBS_OK) return bail(s);
  p->chan_nf = (int*)tmp;
  if ((s = dev_alloc(p, sizeof(nbs::ContractGeom) * n_geom, &tmp, &countdown)) != NBS_OK) return bail(s);
  p->geo = (nbs::ContractGeom*)tmp;
  if ((s = dev_alloc(p, 4, &tmp, &countdown)) != NBS_OK) return bail(s);
  p->nonfinite = (unsigned*)tmp;
  if ((s = dev_alloc(p, 8 * 4, &tmp, &countdown)) != NBS_OK) return bail(s);
  p->queue = (unsigned*)tmp;
  // per geometry: momenta in the order q, -q, q', -q', ...
  std::vector<int*> qorder(n_geom, nullptr);
  for (int i = 0; i < n_geom; ++i) {
    if ((s = dev_alloc(p, p->gw[i].V * 4, &tmp, &countdown)) != NBS_OK) return bail(s);
    qorder[i] = (int*)tmp;
  }
  std::vector<nbs::ContractGeom> geo(n_geom);
  long long b0 = 0;
  for (int i = 0; i < n_geom; ++i) {
    const GeomWork& w = p->gw[i];
    geo[i].Nq = w.Nq;
    geo[i].Ft = w.Ft;
    geo[i].V = (int)w.V;
    geo[i].Lx = w.g.L[0]; geo[i].Ly = w.g.L[1]; geo[i].Lz = w.g.L[2];
    geo[i].t_count = w.g.t_count;
    geo[i].pad = 0;
    geo[i].block0 = b0;
    geo[i].qorder = qorder[i];
    b0 += w.V * w.g.t_count;
  }
  hipError_t e = upload(p, p->chan_nf, nf.data(), nf.size() * 4);
  if (e == hipSuccess) e = upload(p, p->geo, geo.data(), sizeof(nbs::ContractGeom) * n_geom);
  for (int i = 0; i < n_geom && e == hipSuccess; ++i) {
    const int* L = p->gw[i].g.L;
    const int V = (int)p->gw[i].V;
    std::vector<int> order;
    std::vector<char> placed(V, 0);
    for (int q = 0; q < V; ++q) {
      if (placed[q]) continue;
      const int x = q % L[0], y = (q / L[0]) % L[1], z = q / (L[0] * L[1]);
      const int mq = (L[0] - x) % L[0] + L[0] * ((L[1] - y) % L[1] + L[1] * ((L[2] - z) % L[2]));
      order.push_back(q);
      placed[q] = 1;
      if (!placed[mq]) {
        order.push_back(mq);
        placed[mq] = 1;
      }
    }
    e = upload(p, qorder[i], order.data(), (size_t)V * 4);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return bail(NBS_ERR_DEVICE);
  }
  p->n_qt = n_qt;
  if ((s = compile_and_upload(p)) != NBS_OK) return bail(s);
  p->con.geo = p->geo;
  p->con.n_geom = n_geom;
  *out = p;
  return NBS_OK;
}

nbs_status run_plan(nbs_plan p, const void* const* pu, const void* const* pd, const void* const* ps,
                    void* const* F_out, hipStream_t st) {
  nbs_status s = enqueue_build(p, pu, pd, ps, st);
  if (s == NBS_OK) s = enqueue_contract(p, st);
  if (s == NBS_OK) s = enqueue_relsum(p, F_out, st);
  return s;
}

const char* plan_error(const nbs_plan p) { return p ? p->err.c_str() : ""; }

}  // namespace nbs

extern "C" {

nbs_status nbs_plan_create(nbs_plan* out, const nbs_geometry* g, int32_t n_geom, const nbs_channel* ch,
                           int32_t n_ch, nbs_precision prec, int32_t device) {
  return nbs::create_plan(out, g, n_geom, ch, n_ch, prec, device, nullptr, 0, nullptr);
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
  const size_t n = p->gw.size();
  if (!ptrs_ok(prop_u, n) || !ptrs_ok(prop_d, n) || !ptrs_ok(prop_s, n))
    return fail(p, NBS_ERR_INVALID, "null propagator pointer");
  if (hipSetDevice(p->device) != hipSuccess) return fail(p, NBS_ERR_DEVICE, "hipSetDevice");
  const nbs_status s = enqueue_build(p, prop_u, prop_d, prop_s, (hipStream_t)stream);
  if (s != NBS_OK) return s;
  p->stage = ST_BUILT;
  return NBS_OK;
}

nbs_status nbs_contract_channels(nbs_plan p, void* stream) {
  if (!p) return NBS_ERR_INVALID;
  if (p->device < 0) return fail(p, NBS_ERR_STATE, "host-only plan");
  if (p->stage < ST_BUILT) return fail(p, NBS_ERR_STATE, "nbs_build_blocks must come first");
  if (hipSetDevice(p->device) != hipSuccess) return fail(p, NBS_ERR_DEVICE, "hipSetDevice");
  const nbs_status s = enqueue_contract(p, (hipStream_t)stream);
  if (s != NBS_OK) return s;
  p->stage = ST_CONTRACTED;
  return NBS_OK;
}

nbs_status nbs_relative_sum(nbs_plan p, void* const* F_out, void* stream) {
  if (!p) return NBS_ERR_INVALID;
  if (p->device < 0) return fail(p, NBS_ERR_STATE, "host-only plan");
  if (p->stage < ST_CONTRACTED) return fail(p, NBS_ERR_STATE, "nbs_contract_channels must come first");
  if (!ptrs_ok(F_out, p->gw.size())) return fail(p, NBS_ERR_INVALID, "null output pointer");
  if (hipSetDevice(p->device) != hipSuccess) return fail(p, NBS_ERR_DEVICE, "hipSetDevice");
  return enqueue_relsum(p, F_out, (hipStream_t)stream);
}

nbs_status nbs_two_point(nbs_plan p, const nbs_baryon_pair* pairs, int32_t n_pairs, void* const* C_out,
                         void* stream) {
  if (!p) return NBS_ERR_INVALID;
  if (p->device < 0) return fail(p, NBS_ERR_STATE, "host-only plan");
  if (p->stage < ST_BUILT) return fail(p, NBS_ERR_STATE, "nbs_build_blocks must come first");
  if (!pairs || n_pairs < 1 || n_pairs > nbs::kMaxTwoPointPairs)
    return fail(p, NBS_ERR_INVALID, "1 to 8 operator pairs per call");
  if (!ptrs_ok(C_out, p->gw.size())) return fail(p, NBS_ERR_INVALID, "null output pointer");
  const auto& P = p->comp.prog;
  nbs::TwoPointArgs a{};
  a.lay = p->lay;
  a.n_pairs = n_pairs;
  for (int k = 0; k < n_pairs; ++k) {
    const int sink = pairs[k].sink, src = pairs[k].src;
    if (sink < 0 || sink >= NBS_NUM_OPS || src < 0 || src >= NBS_NUM_OPS)
      return fail(p, NBS_ERR_INVALID, "unknown operator");
    int slot = -1;
    for (int s = 0; s < P.n_ops; ++s)
      if (P.op_code[s] == sink) slot = s;
    if (slot < 0) return fail(p, NBS_ERR_INVALID, "the sink operator has no block in this plan");
    const std::vector<nbs::TwoPointTerm> terms = nbs::two_point_terms(sink, src);
    if ((int)terms.size() > nbs::kMaxTwoPointTerms) return fail(p, NBS_ERR_UNSUPPORTED, "too many terms");
    // in the isospin-symmetric limit only canonical blocks exist
    a.slot[k] = p->iso ? P.op_alias[slot] : slot;
    a.slot_coef[k] = p->iso ? P.op_alias_coef[slot] : 1.0;
    nbs::operator_flavour_counts(sink, a.nf[k]);
    a.n_terms[k] = (int)terms.size();
    for (size_t i = 0; i < terms.size(); ++i) {
      a.term_map[k][i] = terms[i].m[0] | (terms[i].m[1] << 2) | (terms[i].m[2] << 4);
      a.term_coef[k][i] = terms[i].coef;
    }
  }
  if (hipSetDevice(p->device) != hipSuccess) return fail(p, NBS_ERR_DEVICE, "hipSetDevice");
  for (size_t g = 0; g < p->gw.size(); ++g) {
    const GeomWork& w = p->gw[g];
    a.Nq = w.Nq;
    a.C = C_out[g];
    a.exps = p->prec == NBS_FP32_MFMA ? w.exps : nullptr;
    a.V = (int)w.V;
    a.t_count = w.g.t_count;
    const nbs_status s = hip_check(p, nbs::launch_two_point(p->prec == NBS_FP64 ? 0 : 1, a, (hipStream_t)stream),
                                   "two-point");
    if (s != NBS_OK) return s;
  }
  return NBS_OK;
}

nbs_status nbs_run_graph(nbs_plan p, const void* const* prop_u, const void* const* prop_d, const void* const* prop_s,
                         void* const* F_out, void* stream) {
  if (!p) return NBS_ERR_INVALID;
  if (p->device < 0) return fail(p, NBS_ERR_STATE, "host-only plan");
  const size_t n = p->gw.size();
  if (!ptrs_ok(prop_u, n) || !ptrs_ok(prop_d, n) || !ptrs_ok(prop_s, n))
    return fail(p, NBS_ERR_INVALID, "null propagator pointer");
  if (!ptrs_ok(F_out, n)) return fail(p, NBS_ERR_INVALID, "null output pointer");
  if (hipSetDevice(p->device) != hipSuccess) return fail(p, NBS_ERR_DEVICE, "hipSetDevice");
  std::vector<const void*> key;
  for (size_t i = 0; i < n; ++i) {
    key.push_back(prop_u[i]);
    key.push_back(prop_d[i]);
    key.push_back(prop_s[i]);
    key.push_back(F_out[i]);
  }
  nbs_status s;
  if (!p->exec || key != p->graph_key) {
    drop_graph(p);
    if (!p->cap_stream &&
        (s = hip_check(p, hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking), "stream")) != NBS_OK)
      return s;
    if ((s = hip_check(p, hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal), "capture")) != NBS_OK)
      return s;
    s = enqueue_build(p, prop_u, prop_d, prop_s, p->cap_stream);
    if (s == NBS_OK) s = enqueue_contract(p, p->cap_stream);
    if (s == NBS_OK) s = enqueue_relsum(p, F_out, p->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
    if (s != NBS_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if ((s = hip_check(p, e, "end capture")) != NBS_OK) return s;
    p->graph = graph;
    if ((s = hip_check(p, hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0), "instantiate")) != NBS_OK) {
      drop_graph(p);
      return s;
    }
    p->graph_key = key;
  }
  if ((s = hip_check(p, hipGraphLaunch(p->exec, (hipStream_t)stream), "graph launch")) != NBS_OK) return s;
  p->stage = ST_CONTRACTED;
  return NBS_OK;
}

nbs_status nbs_plan_autotune(nbs_plan p, const void* const* prop_u, const void* const* prop_d,
                             const void* const* prop_s, void* stream) {
  if (!p) return NBS_ERR_INVALID;
  if (p->device < 0) return fail(p, NBS_ERR_STATE, "host-only plan");
  const size_t n = p->gw.size();
  if (!ptrs_ok(prop_u, n) || !ptrs_ok(prop_d, n) || !ptrs_ok(prop_s, n))
    return fail(p, NBS_ERR_INVALID, "null propagator pointer");
  if (hipSetDevice(p->device) != hipSuccess) return fail(p, NBS_ERR_DEVICE, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  drop_graph(p);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  nbs_status s;
  if ((s = hip_check(p, hipEventCreate(&e0), "event")) != NBS_OK) return s;
  if ((s = hip_check(p, hipEventCreate(&e1), "event")) != NBS_OK) { (void)hipEventDestroy(e0); return s; }
  // time (ms) of fn, run twice after one warm-up
  auto timed = [&](auto fn, float* ms) -> nbs_status {
    nbs_status r = fn();
    if (r != NBS_OK) return r;
    if ((r = hip_check(p, hipEventRecord(e0, st), "event")) != NBS_OK) return r;
    for (int k = 0; k < 2; ++k)
      if ((r = fn()) != NBS_OK) return r;
    if ((r = hip_check(p, hipEventRecord(e1, st), "event")) != NBS_OK) return r;
    if ((r = hip_check(p, hipEventSynchronize(e1), "event")) != NBS_OK) return r;
    return hip_check(p, hipEventElapsedTime(ms, e0, e1), "event");
  };
  auto finish = [&](nbs_status r) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return r;
  };
  // 1. forward transforms: register line kernel or LDS tiles of 512 .. 4096
  //    elements (repeating the in-place transform only costs time; the blocks
  //    are rebuilt at the end)
  struct FftChoice { int cube, plane, line, tile; };
  const FftChoice fft_cands[] = {{1, 1, 1, 1024}, {0, 1, 1, 1024}, {0, 0, 1, 1024}, {0, 0, 0, 512},
                                 {0, 0, 0, 1024}, {0, 0, 0, 2048}, {0, 0, 0, 4096}};
  float best_ms = 0;
  FftChoice best_fft = fft_cands[0];
  bool first = true;
  for (const auto& c : fft_cands) {
    p->tune.fft_cube = c.cube;
    p->tune.fft_plane = c.plane;
    p->tune.fft_line = c.line;
    p->tune.fft_tile = c.tile;
    float ms = 0;
    s = timed([&]() {
      for (auto& w : p->gw) {
        nbs_status r = transform_blocks(p, w, p->comp.prog.n_ops, st);
        if (r != NBS_OK) return r;
      }
      return NBS_OK;
    }, &ms);
    if (s != NBS_OK) return finish(s);
    if (first || ms < best_ms) { best_ms = ms; best_fft = c; first = false; }
  }
  p->tune.fft_cube = best_fft.cube;
  p->tune.fft_plane = best_fft.plane;
  p->tune.fft_line = best_fft.line;
  p->tune.fft_tile = best_fft.tile;
  // 2. contraction: workgroup size (precision form) and index splitting
  if ((s = enqueue_build(p, prop_u, prop_d, prop_s, st)) != NBS_OK) return finish(s);
  // engine 1: matrix-core segments with 16 or 8 wavefronts per workgroup;
  // engine 0: lane teams with their own shapes
  struct ConChoice { int engine, waves, split, mfma; };
  std::vector<ConChoice> con_cands = {{1, 8, 1, 0}, {1, 16, 1, 0}, {0, 8, 1, 0}};
  if (p->prec == NBS_FP32_MFMA) con_cands = {{1, 8, 1, 0}, {1, 16, 1, 0}, {0, 4, 1, 0}};
  ConChoice best_con = con_cands[0];
  first = true;
  const Tuning before = p->tune;
  for (const auto& c : con_cands) {
    p->tune.engine = c.engine;
    if (c.engine == 1) {
      p->tune.seg_waves = c.waves;
      p->tune.waves = before.waves;
    } else {
      p->tune.waves = c.waves;
    }
    p->tune.split = c.split;
    p->tune.mfma = c.mfma;
    if ((s = compile_and_upload(p)) != NBS_OK) return finish(s);
    float ms = 0;
    if ((s = timed([&]() { return enqueue_contract(p, st); }, &ms)) != NBS_OK) return finish(s);
    if (first || ms < best_ms) { best_ms = ms; best_con = c; first = false; }
  }
  p->tune.engine = best_con.engine;
  if (best_con.engine == 1) {
    p->tune.seg_waves = best_con.waves;
    p->tune.waves = before.waves;
  } else {
    p->tune.waves = best_con.waves;
  }
  p->tune.split = best_con.split;
  p->tune.mfma = best_con.mfma;
  // 3. with those: the ranges of groups a workgroup walks
  const int gdefault = p->tune.gchunk;
  int best_g = gdefault;
  for (int gc = 0; gc < 3; ++gc) {
    if (gc == gdefault) continue;
    p->tune.gchunk = gc;
    if ((s = compile_and_upload(p)) != NBS_OK) return finish(s);
    float ms = 0;
    if ((s = timed([&]() { return enqueue_contract(p, st); }, &ms)) != NBS_OK) return finish(s);
    if (ms < best_ms) { best_ms = ms; best_g = gc; }
  }
  p->tune.gchunk = best_g;
  // 4. matrix-core engine: resident workgroups claiming work items, or one
  //    workgroup per item
  if (p->tune.engine == 1) {
    p->tune.persist = 1;
    if ((s = compile_and_upload(p)) != NBS_OK) return finish(s);
    float ms = 0;
    if ((s = timed([&]() { return enqueue_contract(p, st); }, &ms)) != NBS_OK) return finish(s);
    if (!(ms < best_ms)) p->tune.persist = 0;
  } else {
    p->tune.persist = 0;
  }
  if ((s = compile_and_upload(p)) != NBS_OK) return finish(s);
  // leave the plan built with the chosen shapes
  if ((s = enqueue_build(p, prop_u, prop_d, prop_s, st)) != NBS_OK) return finish(s);
  if ((s = hip_check(p, hipStreamSynchronize(st), "sync")) != NBS_OK) return finish(s);
  p->stage = ST_BUILT;
  return finish(NBS_OK);
}

nbs_status nbs_plan_tuning(const nbs_plan p, int32_t out[4]) {
  if (!p || !out) return NBS_ERR_INVALID;
  out[0] = p->tune.fft_line | (p->tune.fft_plane << 1) | (p->tune.fft_cube << 2);
  out[1] = p->tune.fft_tile;
  out[2] = p->tune.engine == 1 ? p->tune.seg_waves : p->tune.waves;
  out[3] = p->tune.split | (p->tune.mfma << 1) | (p->tune.gchunk << 2) | (p->tune.engine << 4) | (p->tune.persist << 5);
  return NBS_OK;
}

nbs_status nbs_plan_set_tuning(nbs_plan p, const int32_t in[4]) {
  if (!p || !in) return NBS_ERR_INVALID;
  const int tile = in[1];
  if (tile != 512 && tile != 1024 && tile != 2048 && tile != 4096) return fail(p, NBS_ERR_INVALID, "fft tile");
  const int waves = in[2];
  const int engine = (in[3] >> 4) & 1;
  const int persist = (in[3] >> 5) & 1;
  if (in[0] < 0 || (in[0] >> 3) != 0 || in[3] < 0 || (in[3] >> 6) != 0)
    return fail(p, NBS_ERR_INVALID, "unknown tuning bits");
  if (persist && engine != 1) return fail(p, NBS_ERR_INVALID, "persistent workgroups need the matrix-core engine");
  if (engine == 1 ? (waves != 8 && waves != 16)
                  : (p->prec == NBS_FP64 ? waves != 8 : (waves != 4 && waves != 8)))
    return fail(p, NBS_ERR_INVALID, "waves");
  if ((in[3] >> 1) & 1 && p->prec != NBS_FP32_MFMA) return fail(p, NBS_ERR_INVALID, "matrix cores need the precision form");
  if (((in[3] >> 2) & 3) > 2) return fail(p, NBS_ERR_INVALID, "group ranges");
  if (p->device >= 0 && hipSetDevice(p->device) != hipSuccess) return fail(p, NBS_ERR_DEVICE, "hipSetDevice");
  if (p->device >= 0 && hipDeviceSynchronize() != hipSuccess) return fail(p, NBS_ERR_DEVICE, "synchronize");
  const Tuning old = p->tune;
  p->tune.fft_line = in[0] & 1;
  p->tune.fft_plane = (in[0] >> 1) & 1;
  p->tune.fft_cube = (in[0] >> 2) & 1;
  p->tune.fft_tile = tile;
  p->tune.engine = engine;
  if (engine == 1) p->tune.seg_waves = waves;
  else p->tune.waves = waves;
  p->tune.split = in[3] & 1;
  p->tune.mfma = (in[3] >> 1) & 1;
  p->tune.gchunk = (in[3] >> 2) & 3;
  p->tune.persist = persist;
  drop_graph(p);
  const nbs_status s = compile_and_upload(p);
  if (s != NBS_OK) {
    p->tune = old;
    (void)compile_and_upload(p);
    return s;
  }
  return NBS_OK;
}

nbs_status nbs_plan_nonfinite(nbs_plan p, int32_t* found) {
  if (!p || !found) return NBS_ERR_INVALID;
  *found = 0;
  if (p->device < 0) return fail(p, NBS_ERR_STATE, "host-only plan");
  if (p->stage < ST_BUILT) return fail(p, NBS_ERR_STATE, "nbs_build_blocks must come first");
  if (hipSetDevice(p->device) != hipSuccess) return fail(p, NBS_ERR_DEVICE, "hipSetDevice");
  nbs_status s;
  if ((s = hip_check(p, hipDeviceSynchronize(), "synchronize")) != NBS_OK) return s;
  unsigned v = 0;
  if ((s = hip_check(p, hipMemcpy(&v, p->nonfinite, 4, hipMemcpyDeviceToHost), "flag read")) != NBS_OK) return s;
  *found = v ? 1 : 0;
  return NBS_OK;
}

nbs_status nbs_plan_destroy(nbs_plan p) {
  if (!p) return NBS_OK;
  if (p->device >= 0 && !p->arena) {
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
  const std::vector<double>* dt = nm == "contrib_coef"       ? &P.contrib_coef
                                  : nm == "op_term_w"        ? &P.op_term_w
                                  : nm == "op_alias_coef"    ? &P.op_alias_coef
                                  : nm == "contrib_coef_iso" ? &P.contrib_coef_iso
                                                             : nullptr;
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
      {"prod_desc", &P.prod_desc}, {"task_lanes", &P.task_lanes}, {"op_alias", &P.op_alias},
      {"group_op1_iso", &P.group_op1_iso}, {"group_op2_iso", &P.group_op2_iso}, {"op_pair", &P.op_pair},
      {"seg_task", &P.seg_task}, {"group_stask", &P.group_stask}, {"prod_ext", &P.prod_ext}, {"contrib_ext", &P.contrib_ext}};
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
