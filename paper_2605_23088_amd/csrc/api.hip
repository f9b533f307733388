// C-ABI entry points (include/yasps.h): context, pattern set-up, and the
// orchestration of one Newton iteration on a single HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/yasps.h"
#include "common.h"
#include "kernels.h"
#include "pattern.h"

using namespace yasps;

namespace {

thread_local std::string g_create_error;

struct Group {
  int type, nfree, begin, end;
};

// Opt-in per-launch event timing, collected at the next host synchronisation.
struct Profiler : LaunchTimer {
  hipStream_t stream = nullptr;
  bool on = false;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  int count[YASPS_K_COUNT] = {};
  double ms[YASPS_K_COUNT] = {};
  int open = -1;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void begin(int cls) override {
    if (!on) return;
    Rec r{cls, get(), get()};
    (void)hipEventRecord(r.a, stream);
    pending.push_back(r);
  }
  void end() override {
    if (!on || pending.empty()) return;
    (void)hipEventRecord(pending.back().b, stream);
  }
  bool kernel_events(int cls, hipEvent_t* start, hipEvent_t* stop) override {
    if (!on) return false;
    Rec r{cls, get(), get()};
    pending.push_back(r);
    *start = r.a;
    *stop = r.b;
    return true;
  }
  // call after the stream has been synchronised
  void collect() {
    for (Rec& r : pending) {
      float t = 0.0f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        count[r.cls]++;
        ms[r.cls] += t;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  void reset() {
    pending.clear();
    for (int k = 0; k < YASPS_K_COUNT; ++k) {
      count[k] = 0;
      ms[k] = 0.0;
    }
  }
  ~Profiler() {
    for (Rec& r : pending) {
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

struct Part {  // device copy of one pattern part
  int nnzb = 0;
  int32_t *rp = nullptr, *ci = nullptr;
};

}  // namespace

struct yasps_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  yasps_problem P{};
  yasps_params prm{};
  int n = 0, nt = 0, nc = 0, nf = 0, nh = 0;
  std::string err;
  std::vector<void*> allocs;      // everything allocated for the static part / workspace
  std::vector<void*> dyn_allocs;  // everything allocated for the current contacts

  // static part
  PartPattern hpat_s;
  Part ps;
  int32_t *spos_t = nullptr, *gpos_t = nullptr, *lead_spos = nullptr, *lead_gpos = nullptr;
  int32_t *cptr_s = nullptr, *gptr_s = nullptr;
  int nblk_s = 0, ngrd_s = 0;
  double *stg_s = nullptr, *gstg_s = nullptr, *vals_s = nullptr;
  float *stg_s32 = nullptr, *vals_s32 = nullptr;
  // cloth (static part): membranes in API order, hinges grouped by free-vertex count
  int32_t *spos_f = nullptr, *gpos_f = nullptr, *spos_h = nullptr, *gpos_h = nullptr, *h_idx = nullptr;
  double* h_rest = nullptr;
  std::vector<Group> hgroups;

  // static share of every full SpMV row (the static-only FullPattern), for the
  // device build of the dynamic part
  int32_t *sf_ptr = nullptr, *sf_col = nullptr, *sf_src = nullptr;
  long long sf_nnz = 0;

  // dynamic part
  PartPattern hpat_d;
  bool hpat_d_current = true;  // false after a device build until yasps_get_pattern downloads it
  int32_t* dslot = nullptr;    // device slot map of a device build [nc][10]
  void* di_arena = nullptr;    // scratch of the device build, grown to the largest build seen
  size_t di_arena_bytes = 0;

  // a second stream for the contact kernels, which run beside the elastic ones
  // during an evaluation (fork / join through the two events)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  Part pd;
  std::vector<Group> groups;
  int32_t *c_idx = nullptr, *spos_c = nullptr, *gpos_c = nullptr, *cptr_d = nullptr, *gptr_d = nullptr,
          *ddiag = nullptr;
  int nblk_d = 0, ngrd_d = 0;
  double *stg_d = nullptr, *gstg_d = nullptr, *vals_d = nullptr, *d_c = nullptr;
  float *stg_d32 = nullptr, *vals_d32 = nullptr;

  // SpMV rows: both triangles of both parts, each entry naming its stored
  // upper block (rebuilt with the contacts; the values are vals_s / vals_d)
  std::vector<void*> full_allocs;
  int32_t *f_rp = nullptr, *f_col = nullptr, *f_src = nullptr;
  float* f_vals32 = nullptr;  // precision form: float32 values per entry, structure of arrays
  // float64: the stored blocks live in one array (static, dynamic, then the
  // transposed copies of the far SpMV entries), reallocated with the rows
  std::vector<void*> val_allocs;
  int32_t* far_src = nullptr;
  int nfar = 0, nnzb_sd = 0;
  long long f_nnz = 0;
  int f_xsplit[PCG_XCDS + 1] = {};

  // shared
  double *grad = nullptr, *minv = nullptr, *parts = nullptr, *scal = nullptr;
  uint32_t* flags = nullptr;
  void* pcg_work = nullptr;
  double *p_dir = nullptr, *x_trial = nullptr, *b_tmp = nullptr;
  double* host_scal = nullptr;  // pinned: [0, 16) scalars and flags, [16, 32) the PCG's polled state
  int pcg_hint = 0;             // iterations of the last PCG solve (sizes the next one's launch batches)
  int nparts_alloc = 0;
  bool evaluated = false;
  bool assembled = false;  // the stored blocks hold the values of the last assembly
  Profiler prof;
};

namespace {

yasps_status fail(yasps_ctx* c, yasps_status s, const std::string& m) {
  if (c)
    c->err = m;
  else
    g_create_error = m;
  return s;
}

#define HIPCHK(ctx, call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail(ctx, YASPS_E_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

template <class T>
hipError_t dalloc(std::vector<void*>& list, T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, n * sizeof(T));
  if (e == hipSuccess) {
    list.push_back(q);
    *p = static_cast<T*>(q);
  }
  return e;
}

template <class T>
hipError_t upload(std::vector<void*>& list, T** p, const std::vector<T>& h, hipStream_t s) {
  hipError_t e = dalloc(list, p, h.size());
  if (e != hipSuccess || h.empty()) return e;
  return hipMemcpyAsync(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

void free_list(std::vector<void*>& list) {
  for (void* p : list) (void)hipFree(p);
  list.clear();
}

int grid_of(int n, int block) { return (n + block - 1) / block; }

yasps_status upload_part(yasps_ctx* c, std::vector<void*>& list, const PartPattern& h, Part& d) {
  d.nnzb = h.nnzb;
  HIPCHK(c, upload(list, &d.rp, h.row_ptr, c->stream));
  HIPCHK(c, upload(list, &d.ci, h.col_idx, c->stream));
  return YASPS_OK;
}

// XCD row ranges of equal work: a row costs its blocks plus about two blocks'
// worth of fixed work (row pointers, the lane-group reduction, the output).
constexpr int XCD_ROW_COST = 2;

// (Re)builds the SpMV matrix layout over the current parts; synchronises the
// stream so the host pattern can go out of scope.
// Float64: marks the far entries of the SpMV rows and (re)allocates the one
// array of stored blocks and far copies that vals_s / vals_d point into (its
// values are written by the next assembly).  The precision form keeps its
// separate arrays.
yasps_status split_far(yasps_ctx* c) {
  c->far_src = nullptr;
  c->nfar = 0;
  const int nd = c->nc ? c->pd.nnzb : 0;
  c->nnzb_sd = c->ps.nnzb + nd;
  if (c->prm.precision == YASPS_MIXED) return YASPS_OK;
  if (c->f_src) {
    auto alloc = [c](size_t bytes) -> void* {
      void* p = nullptr;
      if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
      c->full_allocs.push_back(p);
      return p;
    };
    if (split_far_entries(c->n, c->f_rp, c->f_col, c->f_src, c->ps.nnzb, c->nnzb_sd, FAR_ROWS, &c->far_src,
                          &c->nfar, alloc, c->stream))
      return fail(c, YASPS_E_HIP, "far entries of the SpMV rows");
  }
  std::vector<void*> fresh;
  double* all = nullptr;
  if (dalloc(fresh, &all, 9 * ((size_t)c->nnzb_sd + c->nfar)) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    free_list(fresh);
    return fail(c, YASPS_E_HIP, "array of the stored blocks");
  }
  free_list(c->val_allocs);
  c->val_allocs = fresh;
  c->vals_s = all;
  c->vals_d = nd ? all + 9 * (size_t)c->ps.nnzb : nullptr;
  return YASPS_OK;
}

yasps_status build_full_matrix(yasps_ctx* c) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  free_list(c->full_allocs);
  FullPattern fp;
  build_full(c->n, c->hpat_s, c->nc ? &c->hpat_d : nullptr, fp);
  c->f_nnz = (long long)fp.col.size();
  const long long ROW_COST = XCD_ROW_COST;
  const long long work = c->f_nnz + ROW_COST * c->n;
  int r = 0;
  for (int x = 0; x <= PCG_XCDS; ++x) {
    const long long target = work * x / PCG_XCDS;
    while (r < c->n && (long long)fp.row_ptr[r] + ROW_COST * r < target) ++r;
    c->f_xsplit[x] = x == PCG_XCDS ? c->n : r;
  }
  HIPCHK(c, upload(c->full_allocs, &c->f_rp, fp.row_ptr, c->stream));
  HIPCHK(c, upload(c->full_allocs, &c->f_col, fp.col, c->stream));
  HIPCHK(c, upload(c->full_allocs, &c->f_src, fp.src, c->stream));
  c->f_vals32 = nullptr;
  if (c->prm.precision == YASPS_MIXED) HIPCHK(c, dalloc(c->full_allocs, &c->f_vals32, 9 * (size_t)c->f_nnz));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return split_far(c);
}

// Partials layout: [inertia | tets, membranes, hinge groups | contact energy |
// contact min d | contact active count]
struct PartsLayout {
  int off[6];
};

PartsLayout parts_layout(const yasps_ctx* c) {
  PartsLayout L;
  int nce = 0;
  for (const Group& g : c->groups) nce += grid_of(g.end - g.begin, EVAL_BLOCK);
  int nel = grid_of(c->nt, EVAL_BLOCK) + grid_of(c->nf, EVAL_BLOCK);
  for (const Group& g : c->hgroups) nel += grid_of(g.end - g.begin, EVAL_BLOCK);
  L.off[0] = 0;
  L.off[1] = L.off[0] + grid_of(c->n, EVAL_BLOCK);
  L.off[2] = L.off[1] + nel;
  L.off[3] = L.off[2] + nce;
  L.off[4] = L.off[3] + nce;
  L.off[5] = L.off[4] + nce;
  return L;
}

yasps_status ensure_parts(yasps_ctx* c) {
  const PartsLayout L = parts_layout(c);
  const int need = std::max(L.off[5], 3 * grid_of(std::max(c->n, 1), RED_BLOCK)) + 8;
  if (need <= c->nparts_alloc) return YASPS_OK;
  HIPCHK(c, dalloc(c->allocs, &c->parts, (size_t)need));
  c->nparts_alloc = need;
  return YASPS_OK;
}

SnhArgs snh_args(const yasps_ctx* c, const double* x) {
  SnhArgs a{};
  a.n_free = c->n;
  a.x = x;
  a.x_fixed = c->P.x_fixed;
  a.nt = c->nt;
  a.idx = c->P.tet_idx;
  a.dm_inv = c->P.dm_inv;
  a.vol = c->P.vol;
  a.mu_lam = c->P.mu_lambda;
  a.mu = c->P.mu;
  a.lam = c->P.lambda;
  a.h2 = c->P.h * c->P.h;
  a.spos = c->spos_t;
  a.gpos = c->gpos_t;
  a.blk = c->stg_s;
  a.blk32 = c->stg_s32;
  a.grd = c->gstg_s;
  a.e_part = c->parts + parts_layout(c).off[1];
  a.flags = c->flags;
  return a;
}

MembraneArgs membrane_args(const yasps_ctx* c, const double* x) {
  MembraneArgs a{};
  a.n_free = c->n;
  a.x = x;
  a.x_fixed = c->P.x_fixed;
  a.nf = c->nf;
  a.idx = c->P.tri_idx;
  a.dm_inv = c->P.tri_dm_inv;
  a.area = c->P.tri_area;
  a.mu = c->P.mu_c;
  a.lam = c->P.lambda_c;
  a.thick = c->P.thickness;
  a.h2 = c->P.h * c->P.h;
  a.spos = c->spos_f;
  a.gpos = c->gpos_f;
  a.blk = c->stg_s;
  a.blk32 = c->prm.precision == YASPS_MIXED ? c->stg_s32 : nullptr;
  a.grd = c->gstg_s;
  a.e_part = c->parts + parts_layout(c).off[1] + grid_of(c->nt, EVAL_BLOCK);
  a.flags = c->flags;
  return a;
}

// part_off: partials before this group within the hinge partials
HingeArgs hinge_args(const yasps_ctx* c, const double* x, const Group& g, int part_off) {
  HingeArgs a{};
  a.n_free = c->n;
  a.x = x;
  a.x_fixed = c->P.x_fixed;
  a.begin = g.begin;
  a.end = g.end;
  a.nh = c->nh;
  a.idx = c->h_idx;
  a.rest = c->h_rest;
  a.h2 = c->P.h * c->P.h;
  a.spos = c->spos_h;
  a.gpos = c->gpos_h;
  a.blk = c->stg_s;
  a.blk32 = c->prm.precision == YASPS_MIXED ? c->stg_s32 : nullptr;
  a.grd = c->gstg_s;
  a.e_part = c->parts + parts_layout(c).off[1] + grid_of(c->nt, EVAL_BLOCK) + grid_of(c->nf, EVAL_BLOCK) + part_off;
  a.flags = c->flags;
  return a;
}

InertiaArgs inertia_args(const yasps_ctx* c, const double* x) {
  InertiaArgs a{};
  a.n = c->n;
  a.x = x;
  a.x_tilde = c->P.x_tilde;
  a.mass = c->P.mass;
  a.is_static = c->P.is_static;
  for (int i = 0; i < 3; ++i) a.g[i] = c->P.gravity[i];
  a.spos = c->lead_spos;
  a.gpos = c->lead_gpos;
  a.blk = c->stg_s;
  a.blk32 = c->prm.precision == YASPS_MIXED ? c->stg_s32 : nullptr;
  a.grd = c->gstg_s;
  a.e_part = c->parts;
  a.flags = c->flags;
  return a;
}

ContactArgs contact_args(const yasps_ctx* c, const double* x, const Group& g, int part_off) {
  ContactArgs a{};
  a.n_free = c->n;
  a.x = x;
  a.x_fixed = c->P.x_fixed;
  a.begin = g.begin;
  a.end = g.end;
  a.nc = c->nc;
  a.idx = c->c_idx;
  a.spos = c->spos_c;
  a.gpos = c->gpos_c;
  a.kappa = c->P.kappa;
  a.dhat = c->P.dhat;
  a.barrier = c->prm.barrier;
  a.blk = c->stg_d;
  a.blk32 = c->stg_d32;
  a.grd = c->gstg_d;
  const PartsLayout L = parts_layout(c);
  a.e_part = c->parts + L.off[2] + part_off;
  a.dmin_part = c->parts + L.off[3] + part_off;
  a.nact_part = c->parts + L.off[4] + part_off;
  a.d_out = c->d_c;
  a.flags = c->flags;
  return a;
}

PcgMatrix pcg_matrix(const yasps_ctx* c) {
  PcgMatrix A{};
  A.n = c->n;
  A.rp = c->f_rp;
  A.col = c->f_col;
  A.nnz = c->f_nnz;
  A.minv = c->minv;
  A.src = c->f_src;
  A.vals = c->vals_s;  // float64: the one array of stored blocks and far copies
  A.v32 = c->f_vals32;
  for (int x = 0; x <= PCG_XCDS; ++x) A.xsplit[x] = c->f_xsplit[x];
  return A;
}

yasps_status check_flags(yasps_ctx* c, uint32_t f) {
  if (f & FLAG_NONFINITE) return fail(c, YASPS_E_NONFINITE, "non-finite position or evaluated quantity");
  if (f & FLAG_DOMAIN) return fail(c, YASPS_E_DOMAIN, "a contact stencil has squared distance d <= 0");
  return YASPS_OK;
}

bool valid_ids(const int32_t* idx, int ns, int s, int nv, int nall) {
  for (int a = 0; a < 4; ++a) {
    const int v = idx[a * (size_t)ns + s];
    if (a < nv) {
      if (v < 0 || v >= nall) return false;
      for (int b = 0; b < a; ++b)
        if (idx[b * (size_t)ns + s] == v) return false;
    } else if (v != -1) {
      return false;
    }
  }
  return true;
}

}  // namespace

extern "C" {

const char* yasps_last_error(const yasps_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

void yasps_destroy(yasps_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  free_list(ctx->full_allocs);
  free_list(ctx->dyn_allocs);
  free_list(ctx->val_allocs);
  free_list(ctx->allocs);
  if (ctx->host_scal) (void)hipHostFree(ctx->host_scal);
  if (ctx->di_arena) (void)hipFree(ctx->di_arena);
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
  }
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  delete ctx;
}

yasps_status yasps_create(yasps_ctx** out, void* hip_stream, const yasps_problem* P, const yasps_params* opt) {
  if (!out) return fail(nullptr, YASPS_E_ARG, "out is NULL");
  *out = nullptr;
  if (!P) return fail(nullptr, YASPS_E_ARG, "problem is NULL");
  if (P->n_free < 0 || P->n_fixed < 0 || P->n_tets < 0) return fail(nullptr, YASPS_E_ARG, "negative size");
  if (P->n_free > 0 && (!P->mass || (!P->is_static && !P->x_tilde)))
    return fail(nullptr, YASPS_E_ARG, "mass / x_tilde missing");
  if (P->n_fixed > 0 && !P->x_fixed) return fail(nullptr, YASPS_E_ARG, "x_fixed missing");
  if (P->n_tets > 0 && (!P->tet_idx || !P->dm_inv || !P->vol)) return fail(nullptr, YASPS_E_ARG, "tet arrays missing");
  if (P->n_tris < 0 || P->n_hinges < 0) return fail(nullptr, YASPS_E_ARG, "negative cloth size");
  if (P->n_tris > 0 && (!P->tri_idx || !P->tri_dm_inv || !P->tri_area))
    return fail(nullptr, YASPS_E_ARG, "triangle arrays missing");
  if (P->n_hinges > 0 && (!P->hinge_idx || !P->hinge_rest)) return fail(nullptr, YASPS_E_ARG, "hinge arrays missing");
  if (!(P->dhat > 0.0) || !(P->kappa >= 0.0) || !(P->h > 0.0))
    return fail(nullptr, YASPS_E_ARG, "dhat, kappa and h must be positive");
  yasps_params prm{YASPS_FP64, YASPS_F_SPACE, YASPS_SQLOG, YASPS_INDEX_DEVICE};
  if (opt) prm = *opt;
  if (prm.index_build != YASPS_INDEX_DEVICE && prm.index_build != YASPS_INDEX_HOST)
    return fail(nullptr, YASPS_E_ARG, "unknown index_build");
  if (prm.precision != YASPS_FP64 && prm.precision != YASPS_MIXED)
    return fail(nullptr, YASPS_E_ARG, "unknown precision");
  if (prm.proj != YASPS_F_SPACE) return fail(nullptr, YASPS_E_UNIMPL, "only F-space Neo-Hookean projection is built");
  if (prm.barrier != YASPS_SQLOG && prm.barrier != YASPS_IPC_CLASSIC) return fail(nullptr, YASPS_E_ARG, "unknown barrier");

  yasps_ctx* c = new (std::nothrow) yasps_ctx();
  if (!c) return fail(nullptr, YASPS_E_ARG, "out of host memory");
  auto bail = [&](yasps_status s) {
    g_create_error = c->err;
    yasps_destroy(c);
    return s;
  };
  c->P = *P;
  c->prm = prm;
  c->n = P->n_free;
  c->nt = P->n_tets;
  c->stream = static_cast<hipStream_t>(hip_stream);
  // default priority, non-blocking: ordered against c->stream by events only
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess)
    return bail(fail(c, YASPS_E_HIP, "stream / event creation"));
  if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(c, YASPS_E_HIP, "hipGetDevice failed"));
  {  // device address of the fixed workspace of yasps_pcg_noalloc (once per device; a
     // failure here is reported by that call, which tries again)
    void* sp = nullptr;
    (void)noalloc_scratch(c->device, &sp);
  }
  c->prof.stream = c->stream;

  // validate tets on the host
  std::vector<int32_t> htet((size_t)4 * c->nt);
  if (c->nt) {
    if (hipMemcpy(htet.data(), P->tet_idx, htet.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return bail(fail(c, YASPS_E_HIP, "copying tet_idx failed"));
    const int nall = P->n_free + P->n_fixed;
    for (int t = 0; t < c->nt; ++t)
      if (!valid_ids(htet.data(), c->nt, t, 4, nall))
        return bail(fail(c, YASPS_E_ARG, "tet " + std::to_string(t) + ": vertex id out of range or repeated"));
  }
  // static stencils: tets, then membrane triangles (4th entry -1), then hinges,
  // in API order for the pattern and slot map
  c->nf = P->n_tris;
  c->nh = P->n_hinges;
  const int nt = c->nt, nf = c->nf, nh = c->nh, ns = nt + nf + nh;
  std::vector<int32_t> hst((size_t)4 * ns, -1);
  std::vector<int32_t> htri((size_t)3 * nf), hhin((size_t)4 * nh);
  std::vector<double> hrest((size_t)2 * nh);
  if (nf && hipMemcpy(htri.data(), P->tri_idx, htri.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return bail(fail(c, YASPS_E_HIP, "copying tri_idx failed"));
  if (nh && (hipMemcpy(hhin.data(), P->hinge_idx, hhin.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
             hipMemcpy(hrest.data(), P->hinge_rest, hrest.size() * 8, hipMemcpyDeviceToHost) != hipSuccess))
    return bail(fail(c, YASPS_E_HIP, "copying hinge arrays failed"));
  for (int a = 0; a < 4; ++a) {
    for (int t = 0; t < nt; ++t) hst[(size_t)a * ns + t] = htet[(size_t)a * nt + t];
    if (a < 3)
      for (int f = 0; f < nf; ++f) hst[(size_t)a * ns + nt + f] = htri[(size_t)a * nf + f];
    for (int h = 0; h < nh; ++h) hst[(size_t)a * ns + nt + nf + h] = hhin[(size_t)a * nh + h];
  }
  {
    const int nall = P->n_free + P->n_fixed;
    for (int f = 0; f < nf; ++f)
      if (!valid_ids(hst.data(), ns, nt + f, 3, nall))
        return bail(fail(c, YASPS_E_ARG, "triangle " + std::to_string(f) + ": vertex id out of range or repeated"));
    for (int h = 0; h < nh; ++h)
      if (!valid_ids(hst.data(), ns, nt + nf + h, 4, nall))
        return bail(fail(c, YASPS_E_ARG, "hinge " + std::to_string(h) + ": vertex id out of range or repeated"));
  }
  // hinge storage order: stable by number of free vertices
  std::vector<int> hfree(nh);
  for (int h = 0; h < nh; ++h) {
    int k = 0;
    for (int a = 0; a < 4; ++a) k += hhin[(size_t)a * nh + h] < c->n ? 1 : 0;
    if (k == 0) return bail(fail(c, YASPS_E_ARG, "hinge " + std::to_string(h) + ": no free vertex"));
    hfree[h] = k;
  }
  std::vector<int32_t> horder(nh);
  std::iota(horder.begin(), horder.end(), 0);
  std::stable_sort(horder.begin(), horder.end(), [&](int a, int b) { return hfree[a] < hfree[b]; });
  for (int j = 0; j < nh;) {
    int e = j;
    while (e < nh && hfree[horder[e]] == hfree[horder[j]]) ++e;
    c->hgroups.push_back(Group{0, hfree[horder[j]], j, e});
    j = e;
  }
  build_pattern(c->n, hst.data(), ns, true, c->hpat_s);
  Staging st;
  std::vector<int32_t> order(ns);
  std::iota(order.begin(), order.begin() + nt + nf, 0);
  for (int j = 0; j < nh; ++j) order[nt + nf + j] = nt + nf + horder[j];
  const bool dyn = !P->is_static;
  build_staging(c->n, hst.data(), ns, c->hpat_s, order, dyn, true, st);
  yasps_status s = upload_part(c, c->allocs, c->hpat_s, c->ps);
  if (s) return bail(s);
  {
    FullPattern sf;
    build_full(c->n, c->hpat_s, nullptr, sf);
    c->sf_nnz = (long long)sf.col.size();
    if (upload(c->allocs, &c->sf_ptr, sf.row_ptr, c->stream) != hipSuccess ||
        upload(c->allocs, &c->sf_col, sf.col, c->stream) != hipSuccess ||
        upload(c->allocs, &c->sf_src, sf.src, c->stream) != hipSuccess)
      return bail(fail(c, YASPS_E_HIP, "upload of the static SpMV rows"));
  }
  // per-class staging positions (storage order) and the hinge arrays in storage order
  auto rows = [&](const std::vector<int32_t>& src, int nrows, int j0, int cnt) {
    std::vector<int32_t> out((size_t)nrows * cnt);
    for (int q = 0; q < nrows; ++q)
      for (int j = 0; j < cnt; ++j) out[(size_t)q * cnt + j] = src[(size_t)q * ns + j0 + j];
    return out;
  };
  std::vector<int32_t> hidx_s((size_t)4 * nh);
  std::vector<double> hrest_s((size_t)2 * nh);
  for (int j = 0; j < nh; ++j) {
    for (int a = 0; a < 4; ++a) hidx_s[(size_t)a * nh + j] = hhin[(size_t)a * nh + horder[j]];
    for (int r = 0; r < 2; ++r) hrest_s[(size_t)r * nh + j] = hrest[(size_t)r * nh + horder[j]];
  }
  c->nblk_s = st.nblocks;
  c->ngrd_s = st.ngrads;
#define UP(dst, vec) \
  if (upload(c->allocs, &dst, vec, c->stream) != hipSuccess) return bail(fail(c, YASPS_E_HIP, "upload " #dst));
#define AL(dst, n) \
  if (dalloc(c->allocs, &dst, (size_t)(n)) != hipSuccess) return bail(fail(c, YASPS_E_HIP, "hipMalloc " #dst));
  // (host sources stay alive until the stream synchronisation at the end)
  const std::vector<int32_t> spos_t = rows(st.spos, 10, 0, nt), gpos_t = rows(st.gpos, 4, 0, nt);
  const std::vector<int32_t> spos_f = rows(st.spos, 6, nt, nf), gpos_f = rows(st.gpos, 3, nt, nf);
  const std::vector<int32_t> spos_h = rows(st.spos, 10, nt + nf, nh), gpos_h = rows(st.gpos, 4, nt + nf, nh);
  UP(c->spos_t, spos_t);
  UP(c->gpos_t, gpos_t);
  UP(c->spos_f, spos_f);
  UP(c->gpos_f, gpos_f);
  UP(c->spos_h, spos_h);
  UP(c->gpos_h, gpos_h);
  UP(c->h_idx, hidx_s);
  UP(c->h_rest, hrest_s);
  UP(c->lead_spos, st.lead_spos);
  UP(c->lead_gpos, st.lead_gpos);
  UP(c->cptr_s, st.cptr);
  UP(c->gptr_s, st.gptr);
  if (prm.precision == YASPS_MIXED) {
    AL(c->stg_s32, 9 * (size_t)st.nblocks);
    AL(c->vals_s32, 9 * (size_t)c->hpat_s.nnzb);
  } else {  // vals_s: allocated with the SpMV rows (split_far)
    AL(c->stg_s, 9 * (size_t)st.nblocks);
  }
  AL(c->gstg_s, 3 * (size_t)st.ngrads);
  AL(c->grad, 3 * (size_t)c->n);
  AL(c->minv, 9 * (size_t)c->n);
  AL(c->scal, 64);
  AL(c->flags, 4);
  AL(c->p_dir, 3 * (size_t)c->n);
  AL(c->x_trial, 3 * (size_t)c->n);
  AL(c->b_tmp, 3 * (size_t)c->n);
  {
    char* w = nullptr;
    AL(w, pcg_workspace_bytes(c->n));
    c->pcg_work = w;
  }
  if (hipHostMalloc((void**)&c->host_scal, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return bail(fail(c, YASPS_E_HIP, "hipHostMalloc"));
  s = ensure_parts(c);
  if (s) return bail(s);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(fail(c, YASPS_E_HIP, "stream sync"));
  s = build_full_matrix(c);
  if (s) return bail(s);
#undef UP
#undef AL
  *out = c;
  return YASPS_OK;
}

}  // extern "C"

namespace {

const char* contact_error(int reason) {
  return reason == 1 ? "unknown type" : reason == 2 ? "vertex id out of range, repeated or misplaced" : "no free vertex";
}

// Device build of the dynamic part (build_dynamic_index): the same arrays as the
// host path below, without the round trip through host memory.
yasps_status set_contacts_device(yasps_ctx* c, const yasps_contacts* C) {
  const int nc = C->n_contacts;
  DynIndexIn in{};
  in.n = c->n;
  in.nall = c->P.n_free + c->P.n_fixed;
  in.nc = nc;
  in.type = C->type;
  in.idx = C->idx;
  in.nnzb_s = c->ps.nnzb;
  in.sf_ptr = c->sf_ptr;
  in.sf_col = c->sf_col;
  in.sf_src = c->sf_src;
  in.sf_nnz = c->sf_nnz;
  in.row_cost = XCD_ROW_COST;
  in.arena = c->di_arena;
  in.arena_bytes = c->di_arena_bytes;
  bool oom = false;
  auto alloc_into = [&](std::vector<void*>& list) {
    return [&list, &oom](size_t bytes) -> void* {
      void* p = nullptr;
      if (hipMalloc(&p, bytes) != hipSuccess) {
        oom = true;
        return nullptr;
      }
      list.push_back(p);
      return p;
    };
  };
  // the full rows go to full_allocs, everything else to dyn_allocs
  std::vector<void*> made;
  DynIndexOut o;
  const int r = build_dynamic_index(in, o, alloc_into(made), c->stream);
  if (o.arena_needed > c->di_arena_bytes) {  // the next build with this many contacts needs no allocation
    if (c->di_arena) (void)hipFree(c->di_arena);
    c->di_arena = nullptr;
    c->di_arena_bytes = 0;
    const size_t want = o.arena_needed + o.arena_needed / 4;
    if (hipMalloc(&c->di_arena, want) == hipSuccess) c->di_arena_bytes = want;
  }
  if (r == 1) {
    free_list(made);
    c->nc = 0;
    return fail(c, YASPS_E_ARG, "contact " + std::to_string(o.err_stencil) + ": " + contact_error(o.err_reason));
  }
  if (r != 0 || oom) {
    free_list(made);
    c->nc = 0;
    return fail(c, YASPS_E_HIP, oom ? "out of device memory in the contact index build" : "device build of the contact index");
  }
  for (void* p : made) (o.f_rp == p || o.f_col == p || o.f_src == p ? c->full_allocs : c->dyn_allocs).push_back(p);
  c->nc = nc;
  for (int key = 0, j = 0; key < 32; ++key)
    if (o.gcount[key]) {
      c->groups.push_back(Group{key / 8, key % 8, j, j + o.gcount[key]});
      j += o.gcount[key];
    }
  c->pd.nnzb = o.nnzb;
  c->pd.rp = o.rp;
  c->pd.ci = o.col;
  c->hpat_d.nnzb = o.nnzb;
  c->hpat_d_current = false;
  c->dslot = o.slot;
  c->nblk_d = o.nent;
  c->ngrd_d = o.ngrad;
  c->c_idx = o.sidx;
  c->spos_c = o.spos;
  c->gpos_c = o.gpos;
  c->cptr_d = o.cptr;
  c->gptr_d = o.gptr;
  c->ddiag = o.ddiag;
  if (c->prm.precision == YASPS_MIXED) {
    HIPCHK(c, dalloc(c->dyn_allocs, &c->stg_d32, 9 * (size_t)o.nent));
    HIPCHK(c, dalloc(c->dyn_allocs, &c->vals_d32, 9 * (size_t)o.nnzb));
  } else {  // vals_d: allocated with the SpMV rows (split_far)
    HIPCHK(c, dalloc(c->dyn_allocs, &c->stg_d, 9 * (size_t)o.nent));
  }
  HIPCHK(c, dalloc(c->dyn_allocs, &c->gstg_d, 3 * (size_t)o.ngrad));
  HIPCHK(c, dalloc(c->dyn_allocs, &c->d_c, (size_t)nc));
  yasps_status s = ensure_parts(c);
  if (s) return s;
  // SpMV rows
  c->f_rp = o.f_rp;
  c->f_col = o.f_col;
  c->f_src = o.f_src;
  c->f_nnz = o.f_nnz;
  for (int x = 0; x <= PCG_XCDS; ++x) c->f_xsplit[x] = o.xsplit[x];
  if (c->prm.precision == YASPS_MIXED) HIPCHK(c, dalloc(c->full_allocs, &c->f_vals32, 9 * (size_t)c->f_nnz));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return split_far(c);
}

}  // namespace

extern "C" {

yasps_status yasps_set_contacts(yasps_ctx* c, const yasps_contacts* C) {
  if (!c || !C) return fail(c, YASPS_E_ARG, "NULL argument");
  if (C->n_contacts < 0 || (C->n_contacts > 0 && (!C->type || !C->idx)))
    return fail(c, YASPS_E_ARG, "bad contact arrays");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  free_list(c->dyn_allocs);
  free_list(c->full_allocs);  // rebuilt below, or at the next assembly if this call fails
  c->f_rp = c->f_col = c->f_src = nullptr;
  c->f_vals32 = nullptr;
  c->far_src = nullptr;
  c->nfar = 0;
  c->f_nnz = 0;
  c->groups.clear();
  c->pd = Part{};
  c->hpat_d = PartPattern{};
  c->hpat_d_current = true;
  c->dslot = nullptr;
  c->evaluated = false;
  c->assembled = false;
  const int nc = C->n_contacts;
  if (c->prm.index_build == YASPS_INDEX_DEVICE) return set_contacts_device(c, C);
  std::vector<int32_t> ty(nc), idx((size_t)4 * nc);
  if (nc) {
    HIPCHK(c, hipMemcpy(ty.data(), C->type, (size_t)nc * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(idx.data(), C->idx, idx.size() * 4, hipMemcpyDeviceToHost));
  }
  const int nall = c->P.n_free + c->P.n_fixed;
  static const int NV[4] = {4, 4, 3, 2};
  std::vector<int> key(nc);
  for (int s = 0; s < nc; ++s) {
    if (ty[s] < 0 || ty[s] > 3) {
      c->nc = 0;
      return fail(c, YASPS_E_ARG, "contact " + std::to_string(s) + ": unknown type");
    }
    if (!valid_ids(idx.data(), nc, s, NV[ty[s]], nall)) {
      c->nc = 0;
      return fail(c, YASPS_E_ARG, "contact " + std::to_string(s) + ": vertex id out of range, repeated or misplaced");
    }
    int nf = 0;
    for (int a = 0; a < NV[ty[s]]; ++a) nf += idx[a * (size_t)nc + s] < c->n ? 1 : 0;
    if (nf == 0) {
      c->nc = 0;
      return fail(c, YASPS_E_ARG, "contact " + std::to_string(s) + ": no free vertex");
    }
    // point-triangle stencils against a fixed point get their own group (and
    // kernel): their projection reduces to a 6 x 6 eigenproblem
    const bool pt_fixed_point = ty[s] == 0 && nf == 3 && idx[s] >= c->n;
    key[s] = ty[s] * 8 + (pt_fixed_point ? PT_TRIANGLE_FREE : nf);
  }
  c->nc = nc;
  build_pattern(c->n, idx.data(), nc, false, c->hpat_d);
  // storage order: stable sort by (type, number of free vertices)
  std::vector<int32_t> order(nc);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
  for (int j = 0; j < nc;) {
    int e = j;
    while (e < nc && key[order[e]] == key[order[j]]) ++e;
    c->groups.push_back(Group{key[order[j]] / 8, key[order[j]] % 8, j, e});
    j = e;
  }
  std::vector<int32_t> sidx((size_t)4 * nc);
  for (int j = 0; j < nc; ++j)
    for (int a = 0; a < 4; ++a) sidx[(size_t)a * nc + j] = idx[(size_t)a * nc + order[j]];
  Staging st;
  build_staging(c->n, idx.data(), nc, c->hpat_d, order, false, false, st);
  std::vector<int32_t> ddiag(c->n, -1);
  for (int v = 0; v < c->n; ++v)
    for (int k = c->hpat_d.row_ptr[v]; k < c->hpat_d.row_ptr[v + 1]; ++k)
      if (c->hpat_d.col_idx[k] == v) ddiag[v] = k;
  yasps_status s = upload_part(c, c->dyn_allocs, c->hpat_d, c->pd);
  if (s) return s;
  c->nblk_d = st.nblocks;
  c->ngrd_d = st.ngrads;
  HIPCHK(c, upload(c->dyn_allocs, &c->c_idx, sidx, c->stream));
  HIPCHK(c, upload(c->dyn_allocs, &c->spos_c, st.spos, c->stream));
  HIPCHK(c, upload(c->dyn_allocs, &c->gpos_c, st.gpos, c->stream));
  HIPCHK(c, upload(c->dyn_allocs, &c->cptr_d, st.cptr, c->stream));
  HIPCHK(c, upload(c->dyn_allocs, &c->gptr_d, st.gptr, c->stream));
  HIPCHK(c, upload(c->dyn_allocs, &c->ddiag, ddiag, c->stream));
  if (c->prm.precision == YASPS_MIXED) {
    HIPCHK(c, dalloc(c->dyn_allocs, &c->stg_d32, 9 * (size_t)st.nblocks));
    HIPCHK(c, dalloc(c->dyn_allocs, &c->vals_d32, 9 * (size_t)c->hpat_d.nnzb));
  } else {  // vals_d: allocated with the SpMV rows (split_far)
    HIPCHK(c, dalloc(c->dyn_allocs, &c->stg_d, 9 * (size_t)st.nblocks));
  }
  HIPCHK(c, dalloc(c->dyn_allocs, &c->gstg_d, 3 * (size_t)st.ngrads));
  HIPCHK(c, dalloc(c->dyn_allocs, &c->d_c, (size_t)nc));
  s = ensure_parts(c);
  if (s) return s;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return build_full_matrix(c);
}

namespace {

// Launches every evaluation kernel at x and the final reductions; fills host
// scalars [E_inertia, E_elastic, E_contact, min_d, n_active] and flags.
yasps_status run_eval(yasps_ctx* c, const double* x, int flags, yasps_eval_info* info) {
  const bool exact = (flags & YASPS_EXACT) != 0;
  HIPCHK(c, hipMemsetAsync(c->flags, 0, 4, c->stream));
  if (!c->prof.on && !c->groups.empty()) HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
  c->prof.begin(YASPS_K_INERTIA);
  launch_inertia(inertia_args(c, x), c->stream);
  c->prof.end();
  c->prof.begin(YASPS_K_SNH);
  launch_snh_eval(snh_args(c, x), exact, c->prm.precision == YASPS_MIXED, c->stream);
  c->prof.end();
  if (c->nf || c->nh) {
    c->prof.begin(YASPS_K_CLOTH);
    launch_membrane_eval(membrane_args(c, x), exact, c->stream);
    int hoff = 0;
    for (const Group& g : c->hgroups) {
      launch_hinge_eval(g.nfree, hinge_args(c, x, g, hoff), exact, c->stream);
      hoff += grid_of(g.end - g.begin, EVAL_BLOCK);
    }
    c->prof.end();
  }
  // the contact kernels write only the dynamic staging, their partials and
  // d: they run on the side stream beside the elastic kernels (in sequence
  // while the profiler times kernel classes on the context stream)
  const bool fork = !c->prof.on && !c->groups.empty();
  hipStream_t cs = fork ? c->side : c->stream;
  if (fork) HIPCHK(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
  int off = 0;
  c->prof.begin(YASPS_K_CONTACT);
  for (const Group& g : c->groups) {
    launch_contact_eval(g.type, g.nfree, contact_args(c, x, g, off), exact, cs);
    off += grid_of(g.end - g.begin, EVAL_BLOCK);
  }
  c->prof.end();
  if (fork) {
    HIPCHK(c, hipEventRecord(c->ev_join, c->side));
    HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
  }
  HIPCHK(c, hipGetLastError());
  const PartsLayout L = parts_layout(c);
  const int kinds[5] = {0, 0, 0, 1, 0};
  launch_finalize(5, L.off, c->parts, kinds, c->scal, c->stream);
  HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->host_scal + 8, c->flags, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->prof.collect();
  uint32_t f;
  std::memcpy(&f, c->host_scal + 8, 4);
  const double* h = c->host_scal;
  if (info) {
    info->e_inertia = h[0];
    info->e_elastic = h[1];
    info->e_contact = h[2];
    info->energy = h[0] + h[1] + h[2];
    info->min_d = c->nc ? h[3] : INFINITY;
    info->n_active = (int32_t)h[4];
  }
  c->evaluated = true;
  return check_flags(c, f);
}

// shift > 0 adds shift m_v I to the diagonal blocks (Newton steps with damping).
yasps_status run_assemble(yasps_ctx* c, double shift = 0.0) {
  if (!c->f_rp) {
    const yasps_status s = build_full_matrix(c);
    if (s) return s;
  }
  HIPCHK(c, hipMemsetAsync(c->flags, 0, 4, c->stream));
  c->prof.begin(YASPS_K_ASSEMBLE);
  const bool mixed = c->prm.precision == YASPS_MIXED;
  const bool dyn = c->nc > 0;
  if (mixed) {
    launch_segsum_blocks_f32(c->ps.nnzb, c->nblk_s, c->cptr_s, c->stg_s32, c->vals_s32, c->stream);
    if (dyn) launch_segsum_blocks_f32(c->pd.nnzb, c->nblk_d, c->cptr_d, c->stg_d32, c->vals_d32, c->stream);
  } else {
    launch_segsum_blocks(c->ps.nnzb, c->nblk_s, c->cptr_s, c->stg_s, c->vals_s, c->stream);
    if (dyn) launch_segsum_blocks(c->pd.nnzb, c->nblk_d, c->cptr_d, c->stg_d, c->vals_d, c->stream);
  }
  launch_segsum_grad(c->n, (long long)c->ngrd_s + (dyn ? c->ngrd_d : 0), c->gptr_s, c->gstg_s,
                     dyn ? c->gptr_d : nullptr, dyn ? c->gstg_d : nullptr, c->grad, c->stream);
  launch_add_mass_shift(c->n, c->ps.rp, c->P.mass, shift, c->vals_s, mixed ? c->vals_s32 : nullptr, c->stream);
  if (mixed)
    launch_full_gather_f32(c->f_nnz, c->f_src, c->ps.nnzb, c->vals_s32, dyn ? c->vals_d32 : nullptr, c->f_vals32,
                           c->stream);
  else
    launch_far_gather(c->nfar, c->far_src, c->nnzb_sd, c->vals_s, c->stream);
  c->prof.end();
  c->prof.begin(YASPS_K_BLOCKINV);
  if (mixed)
    launch_block_inverse_f32(c->n, c->ps.rp, c->vals_s32, dyn ? c->ddiag : nullptr, dyn ? c->vals_d32 : nullptr,
                             c->minv, c->flags, c->stream);
  else
    launch_block_inverse(c->n, c->ps.rp, c->vals_s, dyn ? c->ddiag : nullptr, dyn ? c->vals_d : nullptr, c->minv,
                         c->flags, c->stream);
  c->prof.end();
  HIPCHK(c, hipGetLastError());
  c->assembled = true;
  return YASPS_OK;
}

// energy and feasibility at x_trial = x + alpha p; returns E and whether feasible
yasps_status trial_energy(yasps_ctx* c, const double* x0, const double* xt, double* E, bool* feasible) {
  const PartsLayout L = parts_layout(c);
  c->prof.begin(YASPS_K_LINESEARCH);
  InertiaArgs ia = inertia_args(c, xt);
  launch_inertia_energy(ia, c->stream);
  SnhArgs sa = snh_args(c, xt);
  launch_snh_energy(sa, c->stream);
  launch_membrane_energy(membrane_args(c, xt), c->stream);
  int hoff = 0;
  for (const Group& g : c->hgroups) {
    launch_hinge_energy(hinge_args(c, xt, g, hoff), c->stream);
    hoff += grid_of(g.end - g.begin, EVAL_BLOCK);
  }
  int off = 0;
  for (const Group& g : c->groups) {
    ContactArgs ca = contact_args(c, xt, g, off);
    launch_contact_energy(g.type, ca, x0, ca.nact_part, c->stream);  // nact slots reused as "infeasible" counts
    off += grid_of(g.end - g.begin, EVAL_BLOCK);
  }
  c->prof.end();
  HIPCHK(c, hipGetLastError());
  const int kinds[5] = {0, 0, 0, 1, 0};
  launch_finalize(5, L.off, c->parts, kinds, c->scal, c->stream);
  HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->prof.collect();
  const double* h = c->host_scal;
  *E = h[0] + h[1] + h[2];
  *feasible = (h[4] == 0.0) && std::isfinite(*E);
  return YASPS_OK;
}

}  // namespace

yasps_status yasps_eval_stencils(yasps_ctx* c, const double* x, int32_t flags, yasps_eval_info* info) {
  if (!c || !x) return fail(c, YASPS_E_ARG, "NULL argument");
  if (flags != YASPS_PROJECTED && flags != YASPS_EXACT) return fail(c, YASPS_E_ARG, "unknown flags");
  HIPCHK(c, hipSetDevice(c->device));
  return run_eval(c, x, flags, info);
}

yasps_status yasps_assemble_bsr(yasps_ctx* c, yasps_bsr_view* view) {
  if (!c) return fail(c, YASPS_E_ARG, "NULL context");
  if (!c->evaluated) return fail(c, YASPS_E_ARG, "assemble called before any evaluation");
  HIPCHK(c, hipSetDevice(c->device));
  yasps_status s = run_assemble(c);
  if (s) return s;
  HIPCHK(c, hipMemcpyAsync(c->host_scal + 8, c->flags, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  uint32_t f;
  std::memcpy(&f, c->host_scal + 8, 4);
  if (view) {
    view->n_rows = c->n;
    view->nnzb_static = c->ps.nnzb;
    view->nnzb_dynamic = c->nc ? c->pd.nnzb : 0;
    const bool mixed = c->prm.precision == YASPS_MIXED;
    view->row_ptr_s = c->ps.rp;
    view->col_idx_s = c->ps.ci;
    view->values_s = mixed ? (const void*)c->vals_s32 : (const void*)c->vals_s;
    view->row_ptr_d = c->nc ? c->pd.rp : nullptr;
    view->col_idx_d = c->nc ? c->pd.ci : nullptr;
    view->values_d = c->nc ? (mixed ? (const void*)c->vals_d32 : (const void*)c->vals_d) : nullptr;
    view->values_are_f32 = mixed ? 1 : 0;
    view->grad = c->grad;
    view->block_inv = c->minv;
  }
  return check_flags(c, f);
}

}  // extern "C"

namespace {

// yasps_pcg with the solver workspace `work` (the context's, or the fixed
// per-GPU array of yasps_pcg_noalloc).
yasps_status pcg_call(yasps_ctx* c, const double* b, double* x, double rtol, int32_t max_iter, yasps_pcg_info* info,
                      void* work) {
  double rel = 0.0;
  int status = 0;
  const int it = pcg_solve(pcg_matrix(c), b, x, rtol, max_iter, c->prm.precision == YASPS_MIXED, work, &rel,
                           &status, c->stream, &c->prof, c->host_scal + 16, &c->pcg_hint);
  c->prof.collect();
  if (it < 0) return fail(c, YASPS_E_HIP, "pcg launch failed");
  HIPCHK(c, hipGetLastError());
  if (info) {
    info->iters = it;
    info->rel_residual = rel;
    info->status = status;
  }
  if (status == YASPS_E_NOCONV) return fail(c, YASPS_E_NOCONV, "PCG reached max_iter");
  if (status == YASPS_E_BREAKDOWN) return fail(c, YASPS_E_BREAKDOWN, "PCG breakdown: p^T H p <= 0");
  return YASPS_OK;
}

yasps_status pcg_args(yasps_ctx* c, const double* b, double* x, double rtol, int32_t max_iter) {
  if (!c || !b || !x) return fail(c, YASPS_E_ARG, "NULL argument");
  if (!(rtol >= 0.0) || max_iter < 0) return fail(c, YASPS_E_ARG, "bad rtol / max_iter");
  if (!c->evaluated || !c->assembled) return fail(c, YASPS_E_ARG, "pcg called before assembly");
  return YASPS_OK;
}

}  // namespace

extern "C" {

yasps_status yasps_pcg(yasps_ctx* c, const double* b, double* x, double rtol, int32_t max_iter,
                       yasps_pcg_info* info) {
  const yasps_status s = pcg_args(c, b, x, rtol, max_iter);
  if (s) return s;
  HIPCHK(c, hipSetDevice(c->device));
  return pcg_call(c, b, x, rtol, max_iter, info, c->pcg_work);
}

yasps_status yasps_pcg_noalloc(yasps_ctx* c, const double* b, double* x, double rtol, int32_t max_iter,
                               yasps_pcg_info* info) {
  const yasps_status s = pcg_args(c, b, x, rtol, max_iter);
  if (s) return s;
  const size_t need = pcg_workspace_bytes(c->n);
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(c, YASPS_E_ARG, "yasps_pcg_noalloc: " + std::to_string(c->n) + " free vertices need " +
                                    std::to_string(need) + " bytes of solver workspace, more than the fixed " +
                                    std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte array (use yasps_pcg)");
  HIPCHK(c, hipSetDevice(c->device));
  void* work = nullptr;
  HIPCHK(c, noalloc_scratch(c->device, &work));
  return pcg_call(c, b, x, rtol, max_iter, info, work);
}

yasps_status yasps_newton_step(yasps_ctx* c, double* x, const yasps_newton_params* prm, yasps_newton_info* info) {
  if (!c || !x) return fail(c, YASPS_E_ARG, "NULL argument");
  yasps_newton_params p{1e-8, 20000, 40, 1e-4, 0.0, YASPS_PROJECTED, 0.0};
  if (prm) p = *prm;
  if (!(p.shift >= 0.0)) return fail(c, YASPS_E_ARG, "shift must be >= 0");
  if (p.hessian != YASPS_PROJECTED && p.hessian != YASPS_EXACT) return fail(c, YASPS_E_ARG, "unknown hessian mode");
  HIPCHK(c, hipSetDevice(c->device));
  hipEvent_t ev[5];
  for (auto& e : ev) HIPCHK(c, hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() {
      for (int i = 0; i < 5; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  yasps_newton_info ni{};
  HIPCHK(c, hipEventRecord(ev[0], c->stream));
  yasps_eval_info ei{};
  yasps_status s = run_eval(c, x, p.hessian, &ei);
  if (s) return s;
  HIPCHK(c, hipEventRecord(ev[1], c->stream));
  s = run_assemble(c, p.shift);
  if (s) return s;
  HIPCHK(c, hipEventRecord(ev[2], c->stream));
  launch_scale(3 * c->n, c->grad, -1.0, c->b_tmp, c->stream);
  double rel = 0.0;
  int status = 0;
  const int it = pcg_solve(pcg_matrix(c), c->b_tmp, c->p_dir, p.rtol, p.max_iter, c->prm.precision == YASPS_MIXED,
                           c->pcg_work, &rel, &status, c->stream, &c->prof, c->host_scal + 16, &c->pcg_hint);
  c->prof.collect();
  if (it < 0) return fail(c, YASPS_E_HIP, "pcg launch failed");
  HIPCHK(c, hipEventRecord(ev[3], c->stream));
  ni.e0 = ei.energy;
  ni.cg_iters = it;
  ni.cg_rel_residual = rel;
  ni.cg_status = status;
  if (status == YASPS_E_BREAKDOWN) return fail(c, YASPS_E_BREAKDOWN, "PCG breakdown: p^T H p <= 0");
  // max |p_v|, g . p and max |g_v| on the device
  {
    const int nb = grid_of(c->n, RED_BLOCK);
    const int nd = std::min(nb, 1024);
    launch_max_norm3(c->n, c->p_dir, c->parts, nb, c->stream);
    launch_dot(3 * c->n, c->grad, c->p_dir, c->parts + nb, nd, c->stream);
    launch_max_norm3(c->n, c->grad, c->parts + nb + nd, nb, c->stream);
    int off[4] = {0, nb, nb + nd, 2 * nb + nd};
    int kind[3] = {2, 0, 2};
    launch_finalize(3, off, c->parts, kind, c->scal, c->stream);
    HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double pmax = c->host_scal[0];
  const double gp = c->host_scal[1];
  ni.grad_max = c->host_scal[2];
  ni.grad_dot_p = gp;
  if (!(gp < 0.0) && pmax > 0.0) {
    // possible with the exact Hessian away from a minimum: not a descent direction
    ni.e1 = ei.energy;
    if (info) *info = ni;
    return fail(c, YASPS_E_LINESEARCH, "the Newton direction is not a descent direction (g.p >= 0)");
  }
  double alpha = 1.0;
  if (c->nc > 0 && pmax > 0.0) alpha = std::min(1.0, 0.4 * std::sqrt(ei.min_d) / pmax);
  ni.alpha0 = alpha;
  bool accepted = false;
  double E1 = ei.energy;
  int trials = 0;
  for (int k = 0; k <= p.max_halvings; ++k) {
    launch_axpy_to(3 * c->n, x, alpha, c->p_dir, c->x_trial, c->stream);
    double E;
    bool feas;
    ++trials;
    s = trial_energy(c, x, c->x_trial, &E, &feas);
    if (s) return s;
    const bool tie = p.tie_rtol > 0.0 && std::fabs(E - ei.energy) <= p.tie_rtol * std::fabs(ei.energy);
    if (feas && (E <= ei.energy + p.armijo * alpha * gp || tie)) {
      accepted = true;
      E1 = E;
      break;
    }
    alpha *= 0.5;
  }
  if (accepted) HIPCHK(c, hipMemcpyAsync(x, c->x_trial, 3 * (size_t)c->n * 8, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipEventRecord(ev[4], c->stream));
  HIPCHK(c, hipEventSynchronize(ev[4]));
  (void)hipEventElapsedTime(&ni.ms_eval, ev[0], ev[1]);
  (void)hipEventElapsedTime(&ni.ms_assemble, ev[1], ev[2]);
  (void)hipEventElapsedTime(&ni.ms_pcg, ev[2], ev[3]);
  (void)hipEventElapsedTime(&ni.ms_linesearch, ev[3], ev[4]);
  ni.e1 = E1;
  ni.alpha = accepted ? alpha : 0.0;
  ni.step_max = accepted ? alpha * pmax : 0.0;
  ni.ls_trials = trials;
  if (info) *info = ni;
  if (!accepted) return fail(c, YASPS_E_LINESEARCH, "no admissible step after the maximum number of halvings");
  if (status == YASPS_E_NOCONV) return fail(c, YASPS_E_NOCONV, "PCG reached max_iter (step taken with last iterate)");
  return YASPS_OK;
}

yasps_status yasps_get_pattern(yasps_ctx* c, int32_t part, int32_t* row_ptr, int32_t* col_idx, int32_t* slot) {
  if (!c || (part != 0 && part != 1)) return fail(c, YASPS_E_ARG, "bad context or part");
  if (part == 1 && !c->hpat_d_current) {  // device build: copy its pattern and slot map to the host once
    PartPattern& d = c->hpat_d;
    d.row_ptr.resize(c->n + 1);
    d.col_idx.resize(d.nnzb);
    d.slot.resize((size_t)10 * c->nc);
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipMemcpy(d.row_ptr.data(), c->pd.rp, sizeof(int32_t) * (c->n + 1), hipMemcpyDeviceToHost));
    if (d.nnzb) HIPCHK(c, hipMemcpy(d.col_idx.data(), c->pd.ci, sizeof(int32_t) * d.nnzb, hipMemcpyDeviceToHost));
    if (c->nc) HIPCHK(c, hipMemcpy(d.slot.data(), c->dslot, sizeof(int32_t) * 10 * (size_t)c->nc, hipMemcpyDeviceToHost));
    c->hpat_d_current = true;
  }
  const PartPattern& h = part == 0 ? c->hpat_s : c->hpat_d;
  const int n = c->n;
  if (row_ptr) {
    if (h.row_ptr.empty())
      std::fill(row_ptr, row_ptr + n + 1, 0);
    else
      std::copy(h.row_ptr.begin(), h.row_ptr.end(), row_ptr);
  }
  if (col_idx) std::copy(h.col_idx.begin(), h.col_idx.end(), col_idx);
  if (slot) std::copy(h.slot.begin(), h.slot.end(), slot);
  return YASPS_OK;
}

yasps_status yasps_profile_enable(yasps_ctx* c, int32_t enable) {
  if (!c) return fail(c, YASPS_E_ARG, "NULL context");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->prof.collect();
  c->prof.reset();
  c->prof.on = enable != 0;
  return YASPS_OK;
}

yasps_status yasps_profile_query(yasps_ctx* c, int32_t cls, int32_t* launches, double* total_ms) {
  if (!c || cls < 0 || cls >= YASPS_K_COUNT) return fail(c, YASPS_E_ARG, "bad context or kernel class");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->prof.collect();
  if (launches) *launches = c->prof.count[cls];
  if (total_ms) *total_ms = c->prof.ms[cls];
  return YASPS_OK;
}

yasps_status yasps_spmv(yasps_ctx* c, const double* x, double* y) {
  if (!c || !x || !y) return fail(c, YASPS_E_ARG, "NULL argument");
  if (!c->evaluated || !c->assembled) return fail(c, YASPS_E_ARG, "spmv called before assembly");
  HIPCHK(c, hipSetDevice(c->device));
  c->prof.begin(YASPS_K_SPMV);
  launch_spmv(pcg_matrix(c), x, y, c->pcg_work, c->stream);
  c->prof.end();
  HIPCHK(c, hipGetLastError());
  return YASPS_OK;
}

yasps_status yasps_theta_adjoint(yasps_ctx* c, const double* x, const double* lambda, const double* theta,
                                 double* grad_theta) {
  if (!c || !x || !lambda || !theta || !grad_theta) return fail(c, YASPS_E_ARG, "NULL argument");
  HIPCHK(c, hipSetDevice(c->device));
  launch_snh_theta_adjoint(snh_args(c, x), lambda, theta, grad_theta, c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return YASPS_OK;
}

}  // extern "C"
