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
#include "devsort.h"
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

// Device buffer that only grows: reused across contact changes while large enough.
struct GrowBuf {
  void* p = nullptr;
  size_t cap = 0;
  void* ensure(size_t bytes) {
    if (bytes <= cap && p) return p;
    release();
    const size_t want = std::max<size_t>(256, bytes + bytes / 4);
    if (hipMalloc(&p, want) != hipSuccess) {
      p = nullptr;
      return nullptr;
    }
    cap = want;
    return p;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

}  // namespace

struct yasps_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  yasps_problem P{};
  yasps_params prm{};
  int n = 0, nt = 0, nc = 0, nf = 0, nh = 0;  // n: rows of degrees of freedom (nv + 4 nb)
  int nv = 0, nb = 0, nbv = 0;                // free vertices, affine bodies, body vertices
  std::string err;
  std::vector<void*> allocs;      // everything allocated for the static part / workspace

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
  int32_t *spos_bd = nullptr, *gpos_bd = nullptr;  // the bodies' 10 blocks / 4 gradient rows (static staging)
  // SpMV plans of the two parts (spmvplan.hip); their arrays live in the grow-only buffers
  SpmvPart plan_s, plan_d;
  GrowBuf plan_s_buf[PL_COUNT], plan_d_buf[PL_COUNT];

  // dynamic part
  PartPattern hpat_d;
  bool hpat_d_current = true;  // false after a device build until yasps_get_pattern downloads it
  int32_t* dslot = nullptr;    // device slot map of a device build [nc][10]
  void* di_arena = nullptr;    // scratch of the index and plan builds, grown to the largest build seen
  size_t di_arena_bytes = 0;
  // the dynamic part's arrays: grow-only, reused by every contact set that fits
  GrowBuf di_buf[DI_COUNT];
  GrowBuf stg_d_buf, gstg_d_buf, vals_d_buf, d_c_buf;

  // contacts touching affine bodies (third part, built on the host)
  enum { BC_IDX, BC_VPOS, BC_ROWS, BC_SPOS, BC_GPOS, BC_CPTR, BC_GPTR, BC_RP, BC_COL, BC_BDIAG, BC_STG, BC_GSTG,
         BC_VALS, BC_D, BC_PBLK, BC_PGRD, BC_EPS, BC_COUNT };
  GrowBuf bc_buf[BC_COUNT];
  int nbc = 0, nblk_b = 0, ngrd_b = 0;
  std::vector<Group> bgroups;
  PartPattern hpat_b;
  Part pb;
  int32_t *bc_idx = nullptr, *bc_vpos = nullptr, *bc_rows = nullptr, *bc_spos = nullptr, *bc_gpos = nullptr,
          *bc_cptr = nullptr, *bc_gptr = nullptr, *bc_bdiag = nullptr;
  double *stg_b = nullptr, *gstg_b = nullptr, *vals_b = nullptr, *d_b = nullptr, *pos_blk = nullptr,
         *pos_grd = nullptr;
  float *stg_b32 = nullptr, *vals_b32 = nullptr;
  double* bc_eps = nullptr;  // edge-edge mollifier thresholds (storage order) or null
  SpmvPart plan_b;
  GrowBuf plan_b_buf[PL_COUNT];

  // collision surface of the time stepping (proximity search, CCD)
  CdSurface surf{};
  bool has_surface = false;
  std::vector<void*> surf_allocs;
  GrowBuf cd_buf[CD_COUNT];
  CdOutput detected;             // the last proximity search's stencils (device, in cd_buf)
  GrowBuf cd_split[6];           // with bodies: the stencils without / with body vertices (type, idx, eps)
  GrowBuf xt_frame, xs_frame;    // a frame's inertial target and start positions

  // a second stream for the contact kernels, which run beside the elastic ones
  // during an evaluation (fork / join through the two events)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_eval = nullptr;  // after an evaluation's read-back copies (yasps_newton_step)
  Part pd;
  std::vector<Group> groups;
  int32_t *c_idx = nullptr, *spos_c = nullptr, *gpos_c = nullptr, *cptr_d = nullptr, *gptr_d = nullptr,
          *ddiag = nullptr;
  int nblk_d = 0, ngrd_d = 0;
  double *stg_d = nullptr, *gstg_d = nullptr, *vals_d = nullptr, *d_c = nullptr;
  float *stg_d32 = nullptr, *vals_d32 = nullptr;
  double* c_eps = nullptr;  // edge-edge mollifier thresholds (storage order) or null

  // shared
  double *grad = nullptr, *minv = nullptr, *parts = nullptr, *scal = nullptr;
  uint32_t* flags = nullptr;
  GrowBuf pcg_work;             // solver workspace (vectors, partials, SpMV slots)
  double *p_dir = nullptr, *x_trial = nullptr, *b_tmp = nullptr;
  double* host_scal = nullptr;  // pinned: [0, 16) scalars and flags, [16, 32) the PCG's polled state
  int* pin = nullptr;            // pinned read-back scratch of the index, plan and collision builds (PIN_INTS)
  int pcg_hint = 0;             // iterations of the last PCG solve (sizes the next one's launch batches)
  int nparts_alloc = 0;
  bool evaluated = false;
  bool assembled = false;  // the stored blocks hold the values of the last assembly
  Profiler prof;
  hipEvent_t ev[5] = {};        // phase events of yasps_newton_step
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

// Grows the context's index / plan scratch arena to `need` bytes (plus a
// quarter), so the next build of that size allocates no temporaries.
void grow_arena(yasps_ctx* c, size_t need) {
  if (need <= c->di_arena_bytes) return;
  if (c->di_arena) (void)hipFree(c->di_arena);
  c->di_arena = nullptr;
  c->di_arena_bytes = 0;
  const size_t want = need + need / 4;
  if (hipMalloc(&c->di_arena, want) == hipSuccess) c->di_arena_bytes = want;
}

// SpMV plan of one part (0 static, 1 dynamic) into the context's grow-only buffers.
yasps_status build_plan(yasps_ctx* c, int part, const int32_t* rp, const int32_t* col, int nblk, const void* vals) {
  GrowBuf* bufs = part == 0 ? c->plan_s_buf : (part == 1 ? c->plan_d_buf : c->plan_b_buf);
  SpmvPart& out = part == 0 ? c->plan_s : (part == 1 ? c->plan_d : c->plan_b);
  auto alloc = [bufs](int which, size_t bytes) { return bufs[which].ensure(bytes); };
  size_t need = 0;
  const int r = build_spmv_plan(c->n, rp, col, nblk, vals, out, alloc, c->di_arena, c->di_arena_bytes, &need,
                                c->pin, c->stream);
  grow_arena(c, need);
  if (r != 0) {
    out = SpmvPart{};
    return fail(c, YASPS_E_HIP, "building the SpMV plan");
  }
  if (3 * sizeof(double) * (size_t)out.max_entries > spmv_max_lds_bytes()) {
    out = SpmvPart{};
    return fail(c, YASPS_E_ARG, "an SpMV chunk needs more LDS than a workgroup has");
  }
  return YASPS_OK;
}

// The solver workspace for the current plans (grow-only).
yasps_status ensure_pcg_work(yasps_ctx* c) {
  const long long slots =
      (long long)c->plan_s.ntarget + (c->nc ? c->plan_d.ntarget : 0) + (c->nbc ? c->plan_b.ntarget : 0);
  if (!c->pcg_work.ensure(pcg_workspace_bytes(c->n, slots))) return fail(c, YASPS_E_HIP, "hipMalloc of the PCG workspace");
  return YASPS_OK;
}

// Leaves the context without contacts (after a failed or before a new contact set).
void clear_contacts(yasps_ctx* c) {
  c->nc = 0;
  c->groups.clear();
  c->pd = Part{};
  c->plan_d = SpmvPart{};
  c->hpat_d = PartPattern{};
  c->hpat_d_current = true;
  c->dslot = nullptr;
  c->c_idx = c->spos_c = c->gpos_c = c->cptr_d = c->gptr_d = c->ddiag = nullptr;
  c->stg_d = c->gstg_d = c->vals_d = c->d_c = nullptr;
  c->stg_d32 = c->vals_d32 = nullptr;
  c->c_eps = nullptr;
  c->nblk_d = c->ngrd_d = 0;
  c->evaluated = false;
  c->assembled = false;
}

// Partials layout: [inertia: free vertices, bodies | tets, membranes, hinge
// groups, bodies (orthogonality) | contact energy | contact min d | contact
// active count]; the contact segments hold the ordinary contact groups, then
// the body-contact groups.
struct PartsLayout {
  int off[6];
  int body_in, body_or;  // the bodies' inertia and orthogonality partials
  int bc;                // first body-contact partial within each contact segment
};

PartsLayout parts_layout(const yasps_ctx* c) {
  PartsLayout L;
  int nce = 0;
  for (const Group& g : c->groups) nce += grid_of(g.end - g.begin, EVAL_BLOCK);
  L.bc = nce;
  for (const Group& g : c->bgroups) nce += grid_of(g.end - g.begin, EVAL_BLOCK);
  int nel = grid_of(c->nt, EVAL_BLOCK) + grid_of(c->nf, EVAL_BLOCK);
  for (const Group& g : c->hgroups) nel += grid_of(g.end - g.begin, EVAL_BLOCK);
  const int nbp = c->nb ? grid_of(c->nb, EVAL_BLOCK) : 0;
  L.off[0] = 0;
  L.body_in = grid_of(c->nv, EVAL_BLOCK);
  L.off[1] = L.off[0] + L.body_in + nbp;
  L.body_or = L.off[1] + nel;
  nel += nbp;
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
  a.n_free = c->nv;
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
  a.n_free = c->nv;
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
  a.n_free = c->nv;
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
  a.n = c->nv;
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
  a.n_free = c->nv;
  a.x = x;
  a.x_fixed = c->P.x_fixed;
  a.begin = g.begin;
  a.end = g.end;
  a.nc = c->nc;
  a.idx = c->c_idx;
  a.spos = c->spos_c;
  a.gpos = c->gpos_c;
  a.eps = c->c_eps;
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

BodyArgs body_args(const yasps_ctx* c, const double* x) {
  BodyArgs a{};
  a.nv = c->nv;
  a.nb = c->nb;
  a.x = x;
  a.x_tilde = c->P.x_tilde;
  a.M4 = c->P.body_mass;
  a.k = c->P.body_k;
  a.h2 = c->P.h * c->P.h;
  a.is_static = c->P.is_static;
  for (int i = 0; i < 3; ++i) a.g[i] = c->P.gravity[i];
  a.spos = c->spos_bd;
  a.gpos = c->gpos_bd;
  a.blk = c->stg_s;
  a.blk32 = c->prm.precision == YASPS_MIXED ? c->stg_s32 : nullptr;
  a.grd = c->gstg_s;
  const PartsLayout L = parts_layout(c);
  a.e_inertia = c->parts + L.body_in;
  a.e_orth = c->parts + L.body_or;
  a.flags = c->flags;
  return a;
}

// part_off: partials before this group within the body-contact partials
BodyContactArgs body_contact_args(const yasps_ctx* c, const double* x, const Group& g, int part_off) {
  BodyContactArgs a{};
  a.nv = c->nv;
  a.nfix = c->P.n_fixed;
  a.x = x;
  a.x_fixed = c->P.x_fixed;
  a.body_of = c->P.body_of;
  a.body_rest = c->P.body_rest;
  a.begin = g.begin;
  a.end = g.end;
  a.ns = c->nbc;
  a.idx = c->bc_idx;
  a.vpos = c->bc_vpos;
  a.rows = c->bc_rows;
  a.spos = c->bc_spos;
  a.gpos = c->bc_gpos;
  a.eps = c->bc_eps;
  a.kappa = c->P.kappa;
  a.dhat = c->P.dhat;
  a.barrier = c->prm.barrier;
  a.pos_blk = c->pos_blk;
  a.pos_grd = c->pos_grd;
  a.blk = c->stg_b;
  a.blk32 = c->stg_b32;
  a.grd = c->gstg_b;
  const PartsLayout L = parts_layout(c);
  a.e_part = c->parts + L.off[2] + L.bc + part_off;
  a.dmin_part = c->parts + L.off[3] + L.bc + part_off;
  a.nact_part = c->parts + L.off[4] + L.bc + part_off;
  a.d_out = c->d_b;
  a.flags = c->flags;
  return a;
}

PcgMatrix pcg_matrix(const yasps_ctx* c) {
  PcgMatrix A{};
  A.n = c->n;
  A.part[0] = c->plan_s;
  if (c->nc) A.part[1] = c->plan_d;
  if (c->nbc) A.part[2] = c->plan_b;
  A.minv = c->minv;
  A.f32 = c->prm.precision == YASPS_MIXED;
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
  free_list(ctx->allocs);
  for (GrowBuf& b : ctx->bc_buf) b.release();
  for (GrowBuf* set : {ctx->plan_s_buf, ctx->plan_d_buf, ctx->plan_b_buf})
    for (int k = 0; k < PL_COUNT; ++k) set[k].release();
  for (GrowBuf& b : ctx->di_buf) b.release();
  for (GrowBuf& b : ctx->cd_buf) b.release();
  for (GrowBuf& b : ctx->cd_split) b.release();
  free_list(ctx->surf_allocs);
  for (GrowBuf* b : {&ctx->xt_frame, &ctx->xs_frame}) b->release();
  for (GrowBuf* b : {&ctx->stg_d_buf, &ctx->gstg_d_buf, &ctx->vals_d_buf, &ctx->d_c_buf, &ctx->pcg_work}) b->release();
  for (hipEvent_t e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->host_scal) (void)hipHostFree(ctx->host_scal);
  if (ctx->pin) (void)hipHostFree(ctx->pin);
  if (ctx->di_arena) (void)hipFree(ctx->di_arena);
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
  }
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->ev_eval) (void)hipEventDestroy(ctx->ev_eval);
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
  if (P->n_bodies < 0 || P->n_body_verts < 0) return fail(nullptr, YASPS_E_ARG, "negative body size");
  if (P->n_bodies > 0 && (!P->body_mass || !P->body_k || (!P->is_static && !P->x_tilde)))
    return fail(nullptr, YASPS_E_ARG, "body arrays missing");
  if (P->n_body_verts > 0 && (!P->body_of || !P->body_rest || P->n_bodies == 0))
    return fail(nullptr, YASPS_E_ARG, "body vertex arrays missing");
  yasps_params prm{YASPS_FP64, YASPS_F_SPACE, YASPS_SQLOG, YASPS_INDEX_DEVICE};
  if (opt) prm = *opt;
  if (prm.index_build != YASPS_INDEX_DEVICE && prm.index_build != YASPS_INDEX_HOST)
    return fail(nullptr, YASPS_E_ARG, "unknown index_build");
  if (prm.precision != YASPS_FP64 && prm.precision != YASPS_MIXED)
    return fail(nullptr, YASPS_E_ARG, "unknown precision");
  if (prm.proj != YASPS_F_SPACE && prm.proj != YASPS_X_SPACE) return fail(nullptr, YASPS_E_ARG, "unknown proj");
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
  c->nv = P->n_free;
  c->nb = P->n_bodies;
  c->nbv = P->n_body_verts;
  c->n = c->nv + 4 * c->nb;
  c->nt = P->n_tets;
  c->stream = static_cast<hipStream_t>(hip_stream);
  // default priority, non-blocking: ordered against c->stream by events only
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_eval, hipEventDisableTiming) != hipSuccess)
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
  if (c->nbv) {  // every body vertex names a body
    std::vector<int32_t> hb(c->nbv);
    if (hipMemcpy(hb.data(), P->body_of, hb.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return bail(fail(c, YASPS_E_HIP, "copying body_of failed"));
    for (int k = 0; k < c->nbv; ++k)
      if (hb[k] < 0 || hb[k] >= c->nb)
        return bail(fail(c, YASPS_E_ARG, "body vertex " + std::to_string(k) + ": body out of range"));
  }
  // static stencils: tets, then membrane triangles (4th entry -1), then hinges,
  // then the bodies (their 4 rows), in API order for the pattern and slot map;
  // fixed ids move past the body rows (ids >= n have no row)
  c->nf = P->n_tris;
  c->nh = P->n_hinges;
  const int nt = c->nt, nf = c->nf, nh = c->nh, nbd = c->nb, ns = nt + nf + nh + nbd;
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
  for (int a = 0; a < 4; ++a)
    for (int j = 0; j < nt + nf + nh; ++j) {
      int32_t& v = hst[(size_t)a * ns + j];
      if (v >= c->nv) v += 4 * nbd;
    }
  for (int b = 0; b < nbd; ++b)
    for (int a = 0; a < 4; ++a) hst[(size_t)a * ns + nt + nf + nh + b] = c->nv + 4 * b + a;
  // hinge storage order: stable by number of free vertices
  std::vector<int> hfree(nh);
  for (int h = 0; h < nh; ++h) {
    int k = 0;
    for (int a = 0; a < 4; ++a) k += hhin[(size_t)a * nh + h] < c->nv ? 1 : 0;
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
  for (int b = 0; b < nbd; ++b) order[nt + nf + nh + b] = nt + nf + nh + b;
  const bool dyn = !P->is_static;
  build_staging(c->n, hst.data(), ns, c->hpat_s, order, dyn, true, st, 4, c->nv);
  yasps_status s = upload_part(c, c->allocs, c->hpat_s, c->ps);
  if (s) return bail(s);
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
  const std::vector<int32_t> spos_b = rows(st.spos, 10, nt + nf + nh, nbd),
                             gpos_b = rows(st.gpos, 4, nt + nf + nh, nbd);
  UP(c->spos_bd, spos_b);
  UP(c->gpos_bd, gpos_b);
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
  } else {
    AL(c->stg_s, 9 * (size_t)st.nblocks);
    AL(c->vals_s, 9 * (size_t)c->hpat_s.nnzb);
  }
  AL(c->gstg_s, 3 * (size_t)st.ngrads);
  AL(c->grad, 3 * (size_t)c->n);
  AL(c->minv, 9 * (size_t)c->n);
  AL(c->scal, 64);
  AL(c->flags, 4);
  AL(c->p_dir, 3 * (size_t)c->n);
  AL(c->x_trial, 3 * (size_t)c->n);
  AL(c->b_tmp, 3 * (size_t)c->n);
  for (hipEvent_t& e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) return bail(fail(c, YASPS_E_HIP, "hipEventCreate"));
  if (hipHostMalloc((void**)&c->host_scal, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess)
    return bail(fail(c, YASPS_E_HIP, "hipHostMalloc"));
  if (hipHostMalloc((void**)&c->pin, devsort::PIN_INTS * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return bail(fail(c, YASPS_E_HIP, "hipHostMalloc"));
  s = ensure_parts(c);
  if (s) return bail(s);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(fail(c, YASPS_E_HIP, "stream sync"));
  s = build_plan(c, 0, c->ps.rp, c->ps.ci, c->ps.nnzb,
                 prm.precision == YASPS_MIXED ? (const void*)c->vals_s32 : (const void*)c->vals_s);
  if (s) return bail(s);
  s = ensure_pcg_work(c);
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

// After the dynamic pattern and staging layout are on the device: the staged
// and assembled value arrays, the distances, the dynamic SpMV plan and the
// workspace, all in grow-only buffers.  On failure the caller clears the
// contacts.
yasps_status finish_dynamic(yasps_ctx* c) {
  const bool mixed = c->prm.precision == YASPS_MIXED;
  const size_t vsz = mixed ? sizeof(float) : sizeof(double);
  void* stg = c->stg_d_buf.ensure(9 * vsz * (size_t)std::max(c->nblk_d, 1));
  void* vals = c->vals_d_buf.ensure(9 * vsz * (size_t)std::max(c->pd.nnzb, 1));
  c->gstg_d = static_cast<double*>(c->gstg_d_buf.ensure(3 * sizeof(double) * (size_t)std::max(c->ngrd_d, 1)));
  c->d_c = static_cast<double*>(c->d_c_buf.ensure(sizeof(double) * (size_t)std::max(c->nc, 1)));
  if (!stg || !vals || !c->gstg_d || !c->d_c) return fail(c, YASPS_E_HIP, "hipMalloc of the contact arrays");
  if (mixed) {
    c->stg_d32 = static_cast<float*>(stg);
    c->vals_d32 = static_cast<float*>(vals);
  } else {
    c->stg_d = static_cast<double*>(stg);
    c->vals_d = static_cast<double*>(vals);
  }
  yasps_status s = ensure_parts(c);
  if (s) return s;
  s = build_plan(c, 1, c->pd.rp, c->pd.ci, c->pd.nnzb, vals);
  if (s) return s;
  return ensure_pcg_work(c);
}

// Device build of the dynamic part (build_dynamic_index): the same arrays as the
// host path below, without the round trip through host memory.
yasps_status set_contacts_device(yasps_ctx* c, const yasps_contacts* C) {
  const int nc = C->n_contacts;
  DynIndexIn in{};
  in.n = c->nv;
  in.nrows = c->n;
  in.nall = c->P.n_free + c->P.n_fixed;
  in.nc = nc;
  in.type = C->type;
  in.idx = C->idx;
  in.eps = C->ee_eps;
  in.arena = c->di_arena;
  in.arena_bytes = c->di_arena_bytes;
  in.pin = c->pin;
  GrowBuf* bufs = c->di_buf;
  auto alloc = [bufs](int which, size_t bytes) { return bufs[which].ensure(bytes); };
  DynIndexOut o;
  const int r = build_dynamic_index(in, o, alloc, c->stream);
  grow_arena(c, o.arena_needed);  // the next build with this many contacts takes no temporaries
  if (r == 1)
    return fail(c, YASPS_E_ARG, "contact " + std::to_string(o.err_stencil) + ": " + contact_error(o.err_reason));
  if (r != 0) return fail(c, YASPS_E_HIP, "device build of the contact index");
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
  c->c_eps = o.seps;
  c->spos_c = o.spos;
  c->gpos_c = o.gpos;
  c->cptr_d = o.cptr;
  c->gptr_d = o.gptr;
  c->ddiag = o.ddiag;
  return finish_dynamic(c);
}

// Host build of the dynamic part (YASPS_INDEX_HOST), uploaded into the same
// grow-only buffers as the device build.
yasps_status set_contacts_host(yasps_ctx* c, const yasps_contacts* C) {
  const int nc = C->n_contacts;
  std::vector<int32_t> ty(nc), idx((size_t)4 * nc);
  if (nc) {
    HIPCHK(c, hipMemcpy(ty.data(), C->type, (size_t)nc * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(idx.data(), C->idx, idx.size() * 4, hipMemcpyDeviceToHost));
  }
  const int nall = c->P.n_free + c->P.n_fixed;
  static const int NV[4] = {4, 4, 3, 2};
  std::vector<int> key(nc);
  for (int s = 0; s < nc; ++s) {
    if (ty[s] < 0 || ty[s] > 3) return fail(c, YASPS_E_ARG, "contact " + std::to_string(s) + ": unknown type");
    if (!valid_ids(idx.data(), nc, s, NV[ty[s]], nall))
      return fail(c, YASPS_E_ARG, "contact " + std::to_string(s) + ": vertex id out of range, repeated or misplaced");
    int nf = 0;
    for (int a = 0; a < NV[ty[s]]; ++a) nf += idx[a * (size_t)nc + s] < c->nv ? 1 : 0;
    if (nf == 0) return fail(c, YASPS_E_ARG, "contact " + std::to_string(s) + ": no free vertex");
    // point-triangle stencils against a fixed point get their own group (and
    // kernel): their projection reduces to a 6 x 6 eigenproblem
    const bool pt_fixed_point = ty[s] == 0 && nf == 3 && idx[s] >= c->nv;
    key[s] = ty[s] * 8 + (pt_fixed_point ? PT_TRIANGLE_FREE : nf);
  }
  // the pattern over every row: fixed ids move past the affine-body rows
  std::vector<int32_t> ridx(idx);
  for (int32_t& v : ridx)
    if (v >= c->nv) v += c->n - c->nv;
  PartPattern pat;
  build_pattern(c->n, ridx.data(), nc, false, pat);
  // storage order: stable sort by (type, number of free vertices)
  std::vector<int32_t> order(nc);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
  std::vector<Group> groups;
  for (int j = 0; j < nc;) {
    int e = j;
    while (e < nc && key[order[e]] == key[order[j]]) ++e;
    groups.push_back(Group{key[order[j]] / 8, key[order[j]] % 8, j, e});
    j = e;
  }
  std::vector<int32_t> sidx((size_t)4 * nc);
  for (int j = 0; j < nc; ++j)
    for (int a = 0; a < 4; ++a) sidx[(size_t)a * nc + j] = idx[(size_t)a * nc + order[j]];
  std::vector<double> eps, seps;
  if (C->ee_eps) {
    eps.resize(nc);
    seps.resize(nc);
    if (nc) HIPCHK(c, hipMemcpy(eps.data(), C->ee_eps, (size_t)nc * 8, hipMemcpyDeviceToHost));
    for (int j = 0; j < nc; ++j) seps[j] = eps[order[j]];
  }
  Staging st;
  build_staging(c->n, ridx.data(), nc, pat, order, false, false, st);
  std::vector<int32_t> ddiag(c->n, -1);
  for (int v = 0; v < c->n; ++v)
    for (int k = pat.row_ptr[v]; k < pat.row_ptr[v + 1]; ++k)
      if (pat.col_idx[k] == v) ddiag[v] = k;
  auto up = [c](int which, const std::vector<int32_t>& h) -> int32_t* {
    int32_t* d = static_cast<int32_t*>(c->di_buf[which].ensure(sizeof(int32_t) * std::max<size_t>(h.size(), 1)));
    if (d && !h.empty() &&
        hipMemcpyAsync(d, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return nullptr;
    return d;
  };
  c->pd.nnzb = pat.nnzb;
  c->pd.rp = up(DI_RP, pat.row_ptr);
  c->pd.ci = up(DI_COL, pat.col_idx);
  c->c_idx = up(DI_SIDX, sidx);
  c->spos_c = up(DI_SPOS, st.spos);
  c->gpos_c = up(DI_GPOS, st.gpos);
  c->cptr_d = up(DI_CPTR, st.cptr);
  c->gptr_d = up(DI_GPTR, st.gptr);
  c->ddiag = up(DI_DDIAG, ddiag);
  c->c_eps = C->ee_eps ? static_cast<double*>(c->di_buf[DI_EPS].ensure(sizeof(double) * std::max(nc, 1))) : nullptr;
  if (c->c_eps && nc &&
      hipMemcpyAsync(c->c_eps, seps.data(), (size_t)nc * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    c->c_eps = nullptr;
  if (!c->pd.rp || !c->pd.ci || !c->c_idx || !c->spos_c || !c->gpos_c || !c->cptr_d || !c->gptr_d || !c->ddiag ||
      (C->ee_eps && !c->c_eps))
    return fail(c, YASPS_E_HIP, "upload of the contact index");
  HIPCHK(c, hipStreamSynchronize(c->stream));  // the host arrays go out of scope
  c->nc = nc;
  c->groups = std::move(groups);
  c->hpat_d = std::move(pat);
  c->nblk_d = st.nblocks;
  c->ngrd_d = st.ngrads;
  return finish_dynamic(c);
}

// Leaves the context without contacts touching bodies.
void clear_body_contacts(yasps_ctx* c) {
  c->nbc = 0;
  c->bgroups.clear();
  c->pb = Part{};
  c->plan_b = SpmvPart{};
  c->hpat_b = PartPattern{};
  c->bc_eps = nullptr;
  c->nblk_b = c->ngrd_b = 0;
  c->evaluated = false;
  c->assembled = false;
}

// Host build of the body-contact part: row lists (a body's four rows once,
// in vertex order), pattern and slot map over them (up to 8 rows, 36 pairs),
// staging, diagonal positions, then its SpMV plan.
yasps_status set_body_contacts_host(yasps_ctx* c, const yasps_contacts* C) {
  const int ns = C->n_contacts;
  const int nv = c->nv, nfix = c->P.n_fixed, base = nv + nfix, nall = base + c->nbv;
  std::vector<int32_t> ty(ns), idx((size_t)4 * ns), body(c->nbv);
  if (ns) {
    HIPCHK(c, hipMemcpy(ty.data(), C->type, (size_t)ns * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(idx.data(), C->idx, idx.size() * 4, hipMemcpyDeviceToHost));
  }
  if (c->nbv) HIPCHK(c, hipMemcpy(body.data(), c->P.body_of, body.size() * 4, hipMemcpyDeviceToHost));
  static const int NV[4] = {4, 4, 3, 2};
  std::vector<int32_t> rows((size_t)8 * ns, -1), vpos((size_t)4 * ns, -1);
  std::vector<int> key(ns);
  for (int s = 0; s < ns; ++s) {
    const std::string at = "body contact " + std::to_string(s) + ": ";
    if (ty[s] < 0 || ty[s] > 3) return fail(c, YASPS_E_ARG, at + "unknown type");
    if (!valid_ids(idx.data(), ns, s, NV[ty[s]], nall))
      return fail(c, YASPS_E_ARG, at + "vertex id out of range, repeated or misplaced");
    int L = 0, K = 0;
    for (int a = 0; a < NV[ty[s]]; ++a) {
      const int v = idx[(size_t)a * ns + s];
      if (v >= nv && v < base) continue;  // fixed
      ++K;
      int r0[4], nr = 1;
      if (v < nv) {
        r0[0] = v;
      } else {
        const int b = body[v - base];
        nr = 4;
        for (int j = 0; j < 4; ++j) r0[j] = nv + 4 * b + j;
      }
      int first = -1;
      for (int j = 0; j < nr; ++j) {
        int pos = -1;
        for (int q = 0; q < L; ++q)
          if (rows[(size_t)q * ns + s] == r0[j]) pos = q;
        if (pos < 0) {
          if (L == 8) return fail(c, YASPS_E_ARG, at + "more than 8 rows of degrees of freedom");
          rows[(size_t)L * ns + s] = r0[j];
          pos = L++;
        }
        if (j == 0) first = pos;
      }
      vpos[(size_t)a * ns + s] = first;
    }
    if (K == 0) return fail(c, YASPS_E_ARG, at + "no movable vertex");
    key[s] = ty[s] * 8 + K;
  }
  PartPattern pat;
  build_pattern(c->n, rows.data(), ns, false, pat, 8);
  std::vector<int32_t> order(ns);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
  std::vector<Group> groups;
  for (int j = 0; j < ns;) {
    int e = j;
    while (e < ns && key[order[e]] == key[order[j]]) ++e;
    groups.push_back(Group{key[order[j]] / 8, key[order[j]] % 8, j, e});
    j = e;
  }
  Staging st;
  build_staging(c->n, rows.data(), ns, pat, order, false, false, st, 8);
  std::vector<int32_t> sidx((size_t)4 * ns), svpos((size_t)4 * ns), srows((size_t)8 * ns);
  std::vector<double> eps, seps;
  if (C->ee_eps) {
    eps.resize(ns);
    seps.resize(ns);
    if (ns) HIPCHK(c, hipMemcpy(eps.data(), C->ee_eps, (size_t)ns * 8, hipMemcpyDeviceToHost));
    for (int j = 0; j < ns; ++j) seps[j] = eps[order[j]];
  }
  for (int j = 0; j < ns; ++j) {
    for (int a = 0; a < 4; ++a) {
      sidx[(size_t)a * ns + j] = idx[(size_t)a * ns + order[j]];
      svpos[(size_t)a * ns + j] = vpos[(size_t)a * ns + order[j]];
    }
    for (int q = 0; q < 8; ++q) srows[(size_t)q * ns + j] = rows[(size_t)q * ns + order[j]];
  }
  std::vector<int32_t> bdiag(c->n, -1);
  for (int v = 0; v < c->n; ++v)
    for (int k = pat.row_ptr[v]; k < pat.row_ptr[v + 1]; ++k)
      if (pat.col_idx[k] == v) bdiag[v] = k;
  auto up = [c](int which, const std::vector<int32_t>& h) -> int32_t* {
    int32_t* d = static_cast<int32_t*>(c->bc_buf[which].ensure(sizeof(int32_t) * std::max<size_t>(h.size(), 1)));
    if (d && !h.empty() &&
        hipMemcpyAsync(d, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return nullptr;
    return d;
  };
  c->bc_idx = up(yasps_ctx::BC_IDX, sidx);
  c->bc_vpos = up(yasps_ctx::BC_VPOS, svpos);
  c->bc_rows = up(yasps_ctx::BC_ROWS, srows);
  c->bc_spos = up(yasps_ctx::BC_SPOS, st.spos);
  c->bc_gpos = up(yasps_ctx::BC_GPOS, st.gpos);
  c->bc_cptr = up(yasps_ctx::BC_CPTR, st.cptr);
  c->bc_gptr = up(yasps_ctx::BC_GPTR, st.gptr);
  c->pb.rp = up(yasps_ctx::BC_RP, pat.row_ptr);
  c->pb.ci = up(yasps_ctx::BC_COL, pat.col_idx);
  c->bc_bdiag = up(yasps_ctx::BC_BDIAG, bdiag);
  const bool mixed = c->prm.precision == YASPS_MIXED;
  const size_t vsz = mixed ? sizeof(float) : sizeof(double);
  void* stg = c->bc_buf[yasps_ctx::BC_STG].ensure(9 * vsz * (size_t)std::max(st.nblocks, 1));
  void* vals = c->bc_buf[yasps_ctx::BC_VALS].ensure(9 * vsz * (size_t)std::max(pat.nnzb, 1));
  c->gstg_b = static_cast<double*>(c->bc_buf[yasps_ctx::BC_GSTG].ensure(24 * (size_t)std::max(st.ngrads, 1)));
  c->d_b = static_cast<double*>(c->bc_buf[yasps_ctx::BC_D].ensure(8 * (size_t)std::max(ns, 1)));
  c->pos_blk = static_cast<double*>(c->bc_buf[yasps_ctx::BC_PBLK].ensure(8 * 90 * (size_t)std::max(ns, 1)));
  c->pos_grd = static_cast<double*>(c->bc_buf[yasps_ctx::BC_PGRD].ensure(8 * 12 * (size_t)std::max(ns, 1)));
  c->bc_eps = C->ee_eps ? static_cast<double*>(c->bc_buf[yasps_ctx::BC_EPS].ensure(8 * (size_t)std::max(ns, 1)))
                        : nullptr;
  if (c->bc_eps && ns &&
      hipMemcpyAsync(c->bc_eps, seps.data(), (size_t)ns * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    c->bc_eps = nullptr;
  if (!c->bc_idx || !c->bc_vpos || !c->bc_rows || !c->bc_spos || !c->bc_gpos || !c->bc_cptr || !c->bc_gptr ||
      !c->pb.rp || !c->pb.ci || !c->bc_bdiag || !stg || !vals || !c->gstg_b || !c->d_b || !c->pos_blk || !c->pos_grd ||
      (C->ee_eps && !c->bc_eps))
    return fail(c, YASPS_E_HIP, "upload of the body-contact index");
  c->stg_b = mixed ? nullptr : static_cast<double*>(stg);
  c->vals_b = mixed ? nullptr : static_cast<double*>(vals);
  c->stg_b32 = mixed ? static_cast<float*>(stg) : nullptr;
  c->vals_b32 = mixed ? static_cast<float*>(vals) : nullptr;
  HIPCHK(c, hipStreamSynchronize(c->stream));  // the host arrays go out of scope
  c->nbc = ns;
  c->bgroups = std::move(groups);
  c->pb.nnzb = pat.nnzb;
  c->hpat_b = std::move(pat);
  c->nblk_b = st.nblocks;
  c->ngrd_b = st.ngrads;
  yasps_status s = ensure_parts(c);
  if (s) return s;
  s = build_plan(c, 2, c->pb.rp, c->pb.ci, c->pb.nnzb, vals);
  if (s) return s;
  return ensure_pcg_work(c);
}

}  // namespace

extern "C" {

yasps_status yasps_set_body_contacts(yasps_ctx* c, const yasps_contacts* C) {
  if (!c || !C) return fail(c, YASPS_E_ARG, "NULL argument");
  if (C->n_contacts < 0 || (C->n_contacts > 0 && (!C->type || !C->idx)))
    return fail(c, YASPS_E_ARG, "bad contact arrays");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  clear_body_contacts(c);
  const yasps_status s = set_body_contacts_host(c, C);
  if (s) clear_body_contacts(c);  // a rejected or failed set leaves the context without body contacts
  return s;
}

yasps_status yasps_set_contacts(yasps_ctx* c, const yasps_contacts* C) {
  if (!c || !C) return fail(c, YASPS_E_ARG, "NULL argument");
  if (C->n_contacts < 0 || (C->n_contacts > 0 && (!C->type || !C->idx)))
    return fail(c, YASPS_E_ARG, "bad contact arrays");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  clear_contacts(c);
  const yasps_status s =
      c->prm.index_build == YASPS_INDEX_DEVICE ? set_contacts_device(c, C) : set_contacts_host(c, C);
  if (s) clear_contacts(c);  // a rejected or failed set leaves the context without contacts
  return s;
}

namespace {

// Launches every evaluation kernel at x and the final reductions; fills host
// scalars [E_inertia, E_elastic, E_contact, min_d, n_active] and flags.
yasps_status eval_collect(yasps_ctx* c, yasps_eval_info* info, bool drained = true);

// Launches the evaluation and the read-back of its sums and flags; unless
// `defer`, waits for them and returns eval_collect's result, else returns once
// launched (the caller calls eval_collect later).
yasps_status run_eval(yasps_ctx* c, const double* x, int flags, yasps_eval_info* info, bool defer = false) {
  const bool exact = (flags & YASPS_EXACT) != 0;
  HIPCHK(c, hipMemsetAsync(c->flags, 0, 4, c->stream));
  if (!c->prof.on && (!c->groups.empty() || c->nbc)) HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
  c->prof.begin(YASPS_K_INERTIA);
  launch_inertia(inertia_args(c, x), c->stream);
  c->prof.end();
  c->prof.begin(YASPS_K_SNH);
  launch_snh_eval(snh_args(c, x), exact, c->prm.precision == YASPS_MIXED, c->prm.proj == YASPS_X_SPACE, c->stream);
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
  if (c->nb) {
    c->prof.begin(YASPS_K_SNH);
    launch_body_eval(body_args(c, x), exact, c->stream);
    c->prof.end();
  }
  // the contact kernels write only the dynamic staging, their partials and
  // d: they run on the side stream beside the elastic kernels (in sequence
  // while the profiler times kernel classes on the context stream)
  const bool fork = !c->prof.on && (!c->groups.empty() || c->nbc);
  hipStream_t cs = fork ? c->side : c->stream;
  if (fork) HIPCHK(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
  int off = 0;
  c->prof.begin(YASPS_K_CONTACT);
  for (const Group& g : c->groups) {
    launch_contact_eval(g.type, g.nfree, contact_args(c, x, g, off), exact, cs);
    off += grid_of(g.end - g.begin, EVAL_BLOCK);
  }
  // contacts touching bodies: position-space pass per group, then the map to the row lists
  off = 0;
  for (const Group& g : c->bgroups) {
    launch_body_contact_eval(g.type, g.nfree, body_contact_args(c, x, g, off), exact, cs);
    off += grid_of(g.end - g.begin, EVAL_BLOCK);
  }
  if (c->nbc) launch_body_contact_eval(0, -1, body_contact_args(c, x, Group{0, 0, 0, c->nbc}, 0), exact, cs);
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
  HIPCHK(c, hipEventRecord(c->ev_eval, c->stream));
  if (defer) return YASPS_OK;
  return eval_collect(c, info);
}

// The evaluation's energies, minimum distance, active count and status once
// its read-back (ev_eval) has completed.  `drained`: nothing was queued after
// it, so the profiler's records are complete and can be collected.
yasps_status eval_collect(yasps_ctx* c, yasps_eval_info* info, bool drained) {
  HIPCHK(c, hipEventSynchronize(c->ev_eval));
  if (drained) c->prof.collect();
  uint32_t f;
  std::memcpy(&f, c->host_scal + 8, 4);
  const double* h = c->host_scal;
  if (info) {
    info->e_inertia = h[0];
    info->e_elastic = h[1];
    info->e_contact = h[2];
    info->energy = h[0] + h[1] + h[2];
    info->min_d = (c->nc || c->nbc) ? h[3] : INFINITY;
    info->n_active = (int32_t)h[4];
  }
  c->evaluated = true;
  return check_flags(c, f);
}

// shift > 0 adds shift m_v I to the diagonal blocks (Newton steps with damping).
yasps_status run_assemble(yasps_ctx* c, double shift = 0.0) {
  HIPCHK(c, hipMemsetAsync(c->flags, 0, 4, c->stream));
  c->prof.begin(YASPS_K_ASSEMBLE);
  const bool mixed = c->prm.precision == YASPS_MIXED;
  const bool dyn = c->nc > 0;
  const bool bod = c->nbc > 0;
  if (mixed) {
    launch_segsum_blocks_f32(c->ps.nnzb, c->nblk_s, c->cptr_s, c->stg_s32, c->vals_s32, c->stream);
    if (dyn) launch_segsum_blocks_f32(c->pd.nnzb, c->nblk_d, c->cptr_d, c->stg_d32, c->vals_d32, c->stream);
    if (bod) launch_segsum_blocks_f32(c->pb.nnzb, c->nblk_b, c->bc_cptr, c->stg_b32, c->vals_b32, c->stream);
  } else {
    launch_segsum_blocks(c->ps.nnzb, c->nblk_s, c->cptr_s, c->stg_s, c->vals_s, c->stream);
    if (dyn) launch_segsum_blocks(c->pd.nnzb, c->nblk_d, c->cptr_d, c->stg_d, c->vals_d, c->stream);
    if (bod) launch_segsum_blocks(c->pb.nnzb, c->nblk_b, c->bc_cptr, c->stg_b, c->vals_b, c->stream);
  }
  launch_segsum_grad(c->n, (long long)c->ngrd_s + (dyn ? c->ngrd_d : 0) + (bod ? c->ngrd_b : 0), c->gptr_s,
                     c->gstg_s, dyn ? c->gptr_d : nullptr, dyn ? c->gstg_d : nullptr, c->grad, c->stream,
                     bod ? c->bc_gptr : nullptr, bod ? c->gstg_b : nullptr);
  // the damping shift acts on the free vertices' rows (lumped masses)
  launch_add_mass_shift(c->nv, c->ps.rp, c->P.mass, shift, c->vals_s, mixed ? c->vals_s32 : nullptr, c->stream);
  c->prof.end();
  c->prof.begin(YASPS_K_BLOCKINV);
  if (mixed)
    launch_block_inverse_f32(c->n, c->ps.rp, c->vals_s32, dyn ? c->ddiag : nullptr, dyn ? c->vals_d32 : nullptr,
                             c->minv, c->flags, c->stream, bod ? c->bc_bdiag : nullptr, bod ? c->vals_b32 : nullptr);
  else
    launch_block_inverse(c->n, c->ps.rp, c->vals_s, dyn ? c->ddiag : nullptr, dyn ? c->vals_d : nullptr, c->minv,
                         c->flags, c->stream, bod ? c->bc_bdiag : nullptr, bod ? c->vals_b : nullptr);
  c->prof.end();
  HIPCHK(c, hipGetLastError());
  c->assembled = true;
  return YASPS_OK;
}

// energy terms and infeasible count at xt into scal[0..4] (launches only)
yasps_status trial_energy_launch(yasps_ctx* c, const double* x0, const double* xt) {
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
  launch_body_energy(body_args(c, xt), c->stream);
  int off = 0;
  for (const Group& g : c->groups) {
    ContactArgs ca = contact_args(c, xt, g, off);
    launch_contact_energy(g.type, ca, x0, ca.nact_part, c->stream);  // nact slots reused as "infeasible" counts
    off += grid_of(g.end - g.begin, EVAL_BLOCK);
  }
  off = 0;
  for (const Group& g : c->bgroups) {
    BodyContactArgs ba = body_contact_args(c, xt, g, off);
    launch_body_contact_energy(g.type, ba, x0, ba.nact_part, c->stream);
    off += grid_of(g.end - g.begin, EVAL_BLOCK);
  }
  c->prof.end();
  HIPCHK(c, hipGetLastError());
  const int kinds[5] = {0, 0, 0, 1, 0};
  launch_finalize(5, L.off, c->parts, kinds, c->scal, c->stream);
  return YASPS_OK;
}

// energy and feasibility at x_trial = x + alpha p; returns E and whether feasible
yasps_status trial_energy(yasps_ctx* c, const double* x0, const double* xt, double* E, bool* feasible) {
  const yasps_status s = trial_energy_launch(c, x0, xt);
  if (s) return s;
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
    view->nnzb_body = c->nbc ? c->pb.nnzb : 0;
    view->row_ptr_b = c->nbc ? c->pb.rp : nullptr;
    view->col_idx_b = c->nbc ? c->pb.ci : nullptr;
    view->values_b = c->nbc ? (mixed ? (const void*)c->vals_b32 : (const void*)c->vals_b) : nullptr;
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
  return pcg_call(c, b, x, rtol, max_iter, info, c->pcg_work.p);
}

yasps_status yasps_pcg_noalloc(yasps_ctx* c, const double* b, double* x, double rtol, int32_t max_iter,
                               yasps_pcg_info* info) {
  const yasps_status s = pcg_args(c, b, x, rtol, max_iter);
  if (s) return s;
  const long long slots =
      (long long)c->plan_s.ntarget + (c->nc ? c->plan_d.ntarget : 0) + (c->nbc ? c->plan_b.ntarget : 0);
  const size_t need = pcg_workspace_bytes(c->n, slots);
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(c, YASPS_E_ARG, "yasps_pcg_noalloc: " + std::to_string(c->n) + " free vertices and " +
                                    std::to_string(slots) + " SpMV slots need " + std::to_string(need) +
                                    " bytes of solver workspace, more than the fixed " +
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
  hipEvent_t* ev = c->ev;  // created once with the context
  yasps_newton_info ni{};
  HIPCHK(c, hipEventRecord(ev[0], c->stream));
  yasps_eval_info ei{};
  yasps_status s = run_eval(c, x, p.hessian, nullptr, true);
  if (s) return s;
  HIPCHK(c, hipEventRecord(ev[1], c->stream));
  s = run_assemble(c, p.shift);
  if (s) return s;
  HIPCHK(c, hipEventRecord(ev[2], c->stream));
  launch_scale(3 * c->n, c->grad, -1.0, c->b_tmp, c->stream);
  // the evaluation's sums and status (read back while the assembly runs)
  s = eval_collect(c, &ei, false);
  if (s) return s;
  double rel = 0.0;
  int status = 0;
  const int it = pcg_solve(pcg_matrix(c), c->b_tmp, c->p_dir, p.rtol, p.max_iter, c->prm.precision == YASPS_MIXED,
                           c->pcg_work.p, &rel, &status, c->stream, &c->prof, c->host_scal + 16, &c->pcg_hint);
  c->prof.collect();
  if (it < 0) return fail(c, YASPS_E_HIP, "pcg launch failed");
  HIPCHK(c, hipEventRecord(ev[3], c->stream));
  ni.e0 = ei.energy;
  ni.cg_iters = it;
  ni.cg_rel_residual = rel;
  ni.cg_status = status;
  if (status == YASPS_E_BREAKDOWN) return fail(c, YASPS_E_BREAKDOWN, "PCG breakdown: p^T H p <= 0");
  // max |p_v|, g . p and max |g_v| into scal[8..10], the step bound alpha_0
  // into scal[11] and the first trial at x + alpha_0 p, all on the device
  // before one read-back
  const bool contacts = c->nc > 0 || c->nbc > 0;
  {
    const int nb = grid_of(c->n, RED_BLOCK);
    const int nd = std::min(nb, 1024);
    launch_max_norm3(c->n, c->p_dir, c->parts, nb, c->stream);
    launch_dot(3 * c->n, c->grad, c->p_dir, c->parts + nb, nd, c->stream);
    launch_max_norm3(c->n, c->grad, c->parts + nb + nd, nb, c->stream);
    int off[4] = {0, nb, nb + nd, 2 * nb + nd};
    int kind[3] = {2, 0, 2};
    launch_finalize(3, off, c->parts, kind, c->scal + 8, c->stream);
    // the evaluation's minimum distance is still in scal[3]
    launch_step_bound(c->scal + 3, c->scal + 8, contacts ? 1 : 0, c->scal + 11, c->stream);
    launch_axpy_to_dev(3 * c->n, x, c->scal + 11, c->p_dir, c->x_trial, c->stream);
  }
  s = trial_energy_launch(c, x, c->x_trial);
  if (s) return s;
  HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal, 12 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->prof.collect();
  const double* h = c->host_scal;
  const double pmax = h[8];
  const double gp = h[9];
  ni.grad_max = h[10];
  ni.grad_dot_p = gp;
  if (!(gp < 0.0) && pmax > 0.0) {
    // possible with the exact Hessian away from a minimum: not a descent direction
    ni.e1 = ei.energy;
    if (info) *info = ni;
    return fail(c, YASPS_E_LINESEARCH, "the Newton direction is not a descent direction (g.p >= 0)");
  }
  double alpha = h[11];
  ni.alpha0 = alpha;
  bool accepted = false;
  double E1 = ei.energy;
  int trials = 1;
  {
    const double E = h[0] + h[1] + h[2];
    const bool feas = (h[4] == 0.0) && std::isfinite(E);
    const bool tie = p.tie_rtol > 0.0 && std::fabs(E - ei.energy) <= p.tie_rtol * std::fabs(ei.energy);
    if (feas && (E <= ei.energy + p.armijo * alpha * gp || tie)) {
      accepted = true;
      E1 = E;
    }
  }
  for (int k = 1; k <= p.max_halvings && !accepted; ++k) {
    alpha *= 0.5;
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
    }
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
  if (!c || part < 0 || part > 2) return fail(c, YASPS_E_ARG, "bad context or part");
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
  const PartPattern& h = part == 0 ? c->hpat_s : (part == 1 ? c->hpat_d : c->hpat_b);
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
  launch_spmv(pcg_matrix(c), x, y, c->pcg_work.p, c->stream, &c->prof);
  HIPCHK(c, hipGetLastError());
  return YASPS_OK;
}

yasps_status yasps_lm_shift(yasps_ctx* c, double frac, double* out) {
  if (!c || !out) return fail(c, YASPS_E_ARG, "NULL argument");
  if (!(frac >= 0.0)) return fail(c, YASPS_E_ARG, "frac must be >= 0");
  if (!c->evaluated || !c->assembled) return fail(c, YASPS_E_ARG, "lm_shift called before assembly");
  HIPCHK(c, hipSetDevice(c->device));
  const int n = c->nv;  // the free vertices' rows (bodies have no lumped mass)
  if (n == 0) {
    *out = 0.0;
    return YASPS_OK;
  }
  const bool mixed = c->prm.precision == YASPS_MIXED;
  const bool dyn = c->nc > 0, bod = c->nbc > 0;
  // ratios into x_trial, sorted into b_tmp (both (n, 3) work vectors of the context)
  launch_diag_ratio(n, c->ps.rp, mixed ? (const void*)c->vals_s32 : (const void*)c->vals_s, dyn ? c->ddiag : nullptr,
                    dyn ? (mixed ? (const void*)c->vals_d32 : (const void*)c->vals_d) : nullptr,
                    bod ? c->bc_bdiag : nullptr,
                    bod ? (mixed ? (const void*)c->vals_b32 : (const void*)c->vals_b) : nullptr, mixed, c->P.mass,
                    c->x_trial, c->stream);
  HIPCHK(c, hipGetLastError());
  size_t bytes = 0;
  HIPCHK(c, rocprim::radix_sort_keys(nullptr, bytes, c->x_trial, c->b_tmp, (size_t)n, 0u, 64u, c->stream));
  grow_arena(c, bytes);
  if (bytes > c->di_arena_bytes) return fail(c, YASPS_E_HIP, "hipMalloc of the sort scratch");
  HIPCHK(c, rocprim::radix_sort_keys(c->di_arena, bytes, c->x_trial, c->b_tmp, (size_t)n, 0u, 64u, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->host_scal, c->b_tmp + (n - 1) / 2, 2 * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double med = n % 2 ? c->host_scal[0] : 0.5 * (c->host_scal[0] + c->host_scal[1]);
  *out = frac * med;
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

namespace {

CdAlloc cd_alloc(yasps_ctx* c) {
  GrowBuf* bufs = c->cd_buf;
  return [bufs](int which, size_t bytes) { return bufs[which].ensure(bytes); };
}

CdPositions cd_positions(const yasps_ctx* c, const double* x, const double* p = nullptr, double t = 0.0) {
  CdPositions X{};
  X.nv = c->nv;
  X.nfix = c->P.n_fixed;
  X.x = x;
  X.xf = c->P.x_fixed;
  X.body_of = c->nbv ? c->P.body_of : nullptr;
  X.body_rest = c->nbv ? c->P.body_rest : nullptr;
  X.p = p;
  X.t = t;
  return X;
}

// Proximity search at x; the stencils found become the contact set.
yasps_status detect(yasps_ctx* c, const double* x, int32_t* n_out) {
  size_t need = 0;
  const int r = cd_detect(c->surf, cd_positions(c, x), c->P.dhat, cd_alloc(c), c->di_arena, c->di_arena_bytes, &need,
                          c->pin, c->stream, c->detected);
  grow_arena(c, need);
  if (r != 0) {
    c->detected = CdOutput{};
    return r == -2 ? fail(c, YASPS_E_ARG, "proximity search: a box over too many grid cells (a non-finite "
                                          "position, or the cell size far below the primitives)")
                   : fail(c, YASPS_E_HIP, "proximity search");
  }
  if (n_out) *n_out = c->detected.n;
  if (c->nb == 0) {
    yasps_contacts C{c->detected.n, c->detected.type, c->detected.idx, c->surf.len2 ? c->detected.eps : nullptr};
    clear_contacts(c);
    yasps_status s = set_contacts_device(c, &C);
    if (s) clear_contacts(c);
    return s;
  }
  // with bodies: the stencils that reach a body vertex form the body-contact
  // part (host build), the others the dynamic part; each keeps the search's order
  const int n = c->detected.n, base = c->nv + c->P.n_fixed;
  std::vector<int32_t> ty(n), idx((size_t)4 * n);
  std::vector<double> eps(n);
  if (n) {
    HIPCHK(c, hipMemcpy(ty.data(), c->detected.type, (size_t)n * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(idx.data(), c->detected.idx, idx.size() * 4, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(eps.data(), c->detected.eps, (size_t)n * 8, hipMemcpyDeviceToHost));
  }
  std::vector<int> sel[2];
  for (int k = 0; k < n; ++k) {
    bool body = false;
    for (int a = 0; a < 4; ++a) body |= idx[(size_t)a * n + k] >= base;
    sel[body ? 1 : 0].push_back(k);
  }
  yasps_contacts C[2];
  for (int part = 0; part < 2; ++part) {
    const int m = (int)sel[part].size();
    std::vector<int32_t> t(m), i((size_t)4 * m);
    std::vector<double> e(m);
    for (int j = 0; j < m; ++j) {
      const int k = sel[part][j];
      t[j] = ty[k];
      e[j] = eps[k];
      for (int a = 0; a < 4; ++a) i[(size_t)a * m + j] = idx[(size_t)a * n + k];
    }
    GrowBuf* b = c->cd_split + 3 * part;
    int32_t* dt = static_cast<int32_t*>(b[0].ensure(4 * (size_t)std::max(m, 1)));
    int32_t* di = static_cast<int32_t*>(b[1].ensure(16 * (size_t)std::max(m, 1)));
    double* de = static_cast<double*>(b[2].ensure(8 * (size_t)std::max(m, 1)));
    if (!dt || !di || !de) return fail(c, YASPS_E_HIP, "hipMalloc of the split contact lists");
    if (m) {
      HIPCHK(c, hipMemcpy(dt, t.data(), (size_t)m * 4, hipMemcpyHostToDevice));
      HIPCHK(c, hipMemcpy(di, i.data(), i.size() * 4, hipMemcpyHostToDevice));
      HIPCHK(c, hipMemcpy(de, e.data(), (size_t)m * 8, hipMemcpyHostToDevice));
    }
    C[part] = yasps_contacts{m, dt, di, c->surf.len2 ? de : nullptr};
  }
  clear_contacts(c);
  yasps_status s = set_contacts_device(c, &C[0]);
  if (s) {
    clear_contacts(c);
    return s;
  }
  clear_body_contacts(c);
  s = set_body_contacts_host(c, &C[1]);
  if (s) clear_body_contacts(c);
  return s;
}

yasps_status ccd(yasps_ctx* c, const double* x, const double* p, double t_max, double s_ccd, double* t_out) {
  size_t need = 0;
  const int r = cd_ccd(c->surf, cd_positions(c, x, p, t_max), c->P.dhat, t_max, s_ccd, cd_alloc(c), c->di_arena,
                       c->di_arena_bytes, &need, c->pin, c->stream, t_out);
  grow_arena(c, need);
  if (r == -2) return fail(c, YASPS_E_ARG, "CCD: a swept box over too many grid cells (a non-finite position or "
                                           "motion, or the cell size far below the motion)");
  if (r != 0) return fail(c, YASPS_E_HIP, "continuous collision detection");
  return YASPS_OK;
}

// E(x) with the contacts found at x: inertia + elastic terms, plus the
// barrier energy of the proximity search at x.
yasps_status frame_energy(yasps_ctx* c, const double* x, double* E) {
  const PartsLayout L = parts_layout(c);
  c->prof.begin(YASPS_K_LINESEARCH);
  launch_inertia_energy(inertia_args(c, x), c->stream);
  launch_snh_energy(snh_args(c, x), c->stream);
  launch_membrane_energy(membrane_args(c, x), c->stream);
  int hoff = 0;
  for (const Group& g : c->hgroups) {
    launch_hinge_energy(hinge_args(c, x, g, hoff), c->stream);
    hoff += grid_of(g.end - g.begin, EVAL_BLOCK);
  }
  launch_body_energy(body_args(c, x), c->stream);  // the bodies' inertia and orthogonality partials
  c->prof.end();
  HIPCHK(c, hipGetLastError());
  const int kinds[2] = {0, 0};
  launch_finalize(2, L.off, c->parts, kinds, c->scal, c->stream);
  HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  double ec = 0.0;
  size_t need = 0;
  const int r = cd_energy(c->surf, cd_positions(c, x), c->P.dhat, c->P.kappa, c->prm.barrier, cd_alloc(c), c->di_arena,
                          c->di_arena_bytes, &need, c->pin, c->stream, &ec);  // synchronises the stream
  grow_arena(c, need);
  if (r == -2) return fail(c, YASPS_E_ARG, "line search: a box over too many grid cells");
  if (r != 0) return fail(c, YASPS_E_HIP, "contact energy of the proximity search");
  c->prof.collect();
  *E = c->host_scal[0] + c->host_scal[1] + ec;
  return YASPS_OK;
}

}  // namespace

extern "C" {

yasps_status yasps_set_surface(yasps_ctx* c, const yasps_surface* S) {
  if (!c || !S) return fail(c, YASPS_E_ARG, "NULL argument");
  if (S->n_points < 0 || S->n_edges < 0 || S->n_tris < 0 || (S->n_points && !S->points) ||
      (S->n_edges && !S->edges) || (S->n_tris && !S->tris))
    return fail(c, YASPS_E_ARG, "bad surface arrays");
  if (!(S->cell > 0.0)) return fail(c, YASPS_E_ARG, "cell must be > 0");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->has_surface = false;
  free_list(c->surf_allocs);
  const int nall = c->P.n_free + c->P.n_fixed + c->nbv;
  std::vector<int32_t> pts(S->n_points), ed((size_t)2 * S->n_edges), tr((size_t)3 * S->n_tris);
  if (S->n_points) HIPCHK(c, hipMemcpy(pts.data(), S->points, pts.size() * 4, hipMemcpyDeviceToHost));
  if (S->n_edges) HIPCHK(c, hipMemcpy(ed.data(), S->edges, ed.size() * 4, hipMemcpyDeviceToHost));
  if (S->n_tris) HIPCHK(c, hipMemcpy(tr.data(), S->tris, tr.size() * 4, hipMemcpyDeviceToHost));
  auto bad = [nall](int v) { return v < 0 || v >= nall; };
  for (int32_t v : pts)
    if (bad(v)) return fail(c, YASPS_E_ARG, "surface point id out of range");
  for (int j = 0; j < S->n_edges; ++j)
    if (bad(ed[j]) || bad(ed[(size_t)S->n_edges + j]) || ed[j] == ed[(size_t)S->n_edges + j])
      return fail(c, YASPS_E_ARG, "surface edge " + std::to_string(j) + ": bad vertex ids");
  for (int j = 0; j < S->n_tris; ++j) {
    const int a = tr[j], b = tr[(size_t)S->n_tris + j], d = tr[2 * (size_t)S->n_tris + j];
    if (bad(a) || bad(b) || bad(d) || a == b || b == d || a == d)
      return fail(c, YASPS_E_ARG, "surface triangle " + std::to_string(j) + ": bad vertex ids");
  }
  CdSurface& D = c->surf;
  D = CdSurface{};
  D.np = S->n_points;
  D.ne = S->n_edges;
  D.nt = S->n_tris;
  D.cell = S->cell;
  int32_t *dp = nullptr, *de = nullptr, *dt = nullptr;
  HIPCHK(c, upload(c->surf_allocs, &dp, pts, c->stream));
  HIPCHK(c, upload(c->surf_allocs, &de, ed, c->stream));
  HIPCHK(c, upload(c->surf_allocs, &dt, tr, c->stream));
  D.points = dp;
  D.edges = de;
  D.tris = dt;
  if (S->edge_rest_len2) {
    double* dl = nullptr;
    HIPCHK(c, dalloc(c->surf_allocs, &dl, (size_t)std::max(S->n_edges, 1)));
    if (S->n_edges)
      HIPCHK(c, hipMemcpyAsync(dl, S->edge_rest_len2, (size_t)S->n_edges * 8, hipMemcpyDeviceToDevice, c->stream));
    D.len2 = dl;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->has_surface = true;
  return YASPS_OK;
}

yasps_status yasps_detect(yasps_ctx* c, const double* x, int32_t* n_contacts) {
  if (!c || !x) return fail(c, YASPS_E_ARG, "NULL argument");
  if (!c->has_surface) return fail(c, YASPS_E_ARG, "no collision surface (yasps_set_surface)");
  HIPCHK(c, hipSetDevice(c->device));
  return detect(c, x, n_contacts);
}

yasps_status yasps_get_detected(yasps_ctx* c, int32_t* type, int32_t* idx, double* ee_eps) {
  if (!c) return fail(c, YASPS_E_ARG, "NULL context");
  HIPCHK(c, hipSetDevice(c->device));
  const CdOutput& o = c->detected;
  if (o.n == 0) return YASPS_OK;
  if (type) HIPCHK(c, hipMemcpy(type, o.type, (size_t)o.n * 4, hipMemcpyDeviceToHost));
  if (idx) HIPCHK(c, hipMemcpy(idx, o.idx, 4 * (size_t)o.n * 4, hipMemcpyDeviceToHost));
  if (ee_eps) HIPCHK(c, hipMemcpy(ee_eps, o.eps, (size_t)o.n * 8, hipMemcpyDeviceToHost));
  return YASPS_OK;
}

yasps_status yasps_ccd(yasps_ctx* c, const double* x, const double* p, double t_max, double s, double* t_out) {
  if (!c || !x || !p || !t_out) return fail(c, YASPS_E_ARG, "NULL argument");
  if (!c->has_surface) return fail(c, YASPS_E_ARG, "no collision surface (yasps_set_surface)");
  if (!(t_max >= 0.0) || !(s > 0.0 && s < 1.0)) return fail(c, YASPS_E_ARG, "need t_max >= 0 and 0 < s < 1");
  HIPCHK(c, hipSetDevice(c->device));
  return ccd(c, x, p, t_max, s, t_out);
}

yasps_status yasps_frame(yasps_ctx* c, double* x, double* v, const yasps_frame_params* prm, yasps_frame_info* info) {
  if (!c || !x || !v) return fail(c, YASPS_E_ARG, "NULL argument");
  yasps_frame_params fp{1e-2, 50, 1e-8, 20000, 1e-4, 40, 0.1};
  if (prm) fp = *prm;
  if (!(fp.tol > 0.0) || fp.max_newton < 1 || !(fp.ccd_s > 0.0 && fp.ccd_s < 1.0))
    return fail(c, YASPS_E_ARG, "need tol > 0, max_newton >= 1, 0 < ccd_s < 1");
  if (c->P.is_static) return fail(c, YASPS_E_ARG, "time stepping needs the dynamic form (is_static = 0)");
  if (!c->has_surface) return fail(c, YASPS_E_ARG, "no collision surface (yasps_set_surface)");
  HIPCHK(c, hipSetDevice(c->device));
  const double h = c->P.h;
  const size_t bytes = 3 * (size_t)c->n * sizeof(double);
  double* xt = static_cast<double*>(c->xt_frame.ensure(std::max<size_t>(bytes, 8)));
  double* xs = static_cast<double*>(c->xs_frame.ensure(std::max<size_t>(bytes, 8)));
  if (!xt || !xs) return fail(c, YASPS_E_HIP, "hipMalloc of the frame buffers");
  launch_frame_tilde(c->nv, c->n, x, v, h, c->P.gravity, xt, c->stream);
  HIPCHK(c, hipMemcpyAsync(xs, x, bytes, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipGetLastError());
  // the frame's inertial target replaces the problem's for its duration
  struct Restore {
    yasps_ctx* c;
    const double* keep;
    ~Restore() { c->P.x_tilde = keep; }
  } restore{c, c->P.x_tilde};
  c->P.x_tilde = xt;
  yasps_frame_info fi{};
  fi.alpha_min = 1.0;
  hipEvent_t* ev = c->ev;
  float ms;
  yasps_status s = YASPS_OK;
  for (int it = 0; it < fp.max_newton; ++it) {
    HIPCHK(c, hipEventRecord(ev[0], c->stream));
    int32_t nc = 0;
    s = detect(c, x, &nc);
    if (s) return s;
    fi.n_contacts_max = std::max(fi.n_contacts_max, nc);
    HIPCHK(c, hipEventRecord(ev[1], c->stream));
    yasps_eval_info ei{};
    s = run_eval(c, x, YASPS_PROJECTED, &ei);
    if (s) return s;
    if (it == 0) fi.e_begin = ei.energy;
    fi.e_end = ei.energy;
    s = run_assemble(c);
    if (s) return s;
    launch_scale(3 * c->n, c->grad, -1.0, c->b_tmp, c->stream);
    double rel = 0.0;
    int status = 0;
    const int cg = pcg_solve(pcg_matrix(c), c->b_tmp, c->p_dir, fp.rtol, fp.max_iter, c->prm.precision == YASPS_MIXED,
                             c->pcg_work.p, &rel, &status, c->stream, &c->prof, c->host_scal + 16, &c->pcg_hint);
    c->prof.collect();
    if (cg < 0) return fail(c, YASPS_E_HIP, "pcg launch failed");
    if (status == YASPS_E_BREAKDOWN) return fail(c, YASPS_E_BREAKDOWN, "PCG breakdown: p^T H p <= 0");
    fi.cg_iters += cg;
    {
      const int nb = grid_of(c->n, RED_BLOCK);
      const int nd = std::min(nb, 1024);
      launch_max_norm3(c->n, c->p_dir, c->parts, nb, c->stream);
      launch_dot(3 * c->n, c->grad, c->p_dir, c->parts + nb, nd, c->stream);
      int off[3] = {0, nb, nb + nd};
      int kind[2] = {2, 0};
      launch_finalize(2, off, c->parts, kind, c->scal, c->stream);
      HIPCHK(c, hipMemcpyAsync(c->host_scal, c->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipEventRecord(ev[2], c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double pmax = c->host_scal[0], gp = c->host_scal[1];
    (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
    fi.ms_detect += ms;
    (void)hipEventElapsedTime(&ms, ev[1], ev[2]);
    fi.ms_newton += ms;
    if (pmax / h < fp.tol) {  // the paper's stop rule: largest displacement per time step
      fi.converged = 1;
      break;
    }
    if (!(gp < 0.0)) return fail(c, YASPS_E_LINESEARCH, "the Newton direction is not a descent direction");
    ++fi.newton_iters;
    double alpha = 1.0;
    s = ccd(c, x, c->p_dir, 1.0, fp.ccd_s, &alpha);
    if (s) return s;
    HIPCHK(c, hipEventRecord(ev[3], c->stream));
    HIPCHK(c, hipEventSynchronize(ev[3]));
    ms = 0.0f;
    (void)hipEventElapsedTime(&ms, ev[2], ev[3]);
    fi.ms_ccd += ms;
    bool accepted = false;
    for (int k = 0; k <= fp.max_halvings; ++k) {
      launch_axpy_to(3 * c->n, x, alpha, c->p_dir, c->x_trial, c->stream);
      double E = 0.0;
      ++fi.ls_trials;
      s = frame_energy(c, c->x_trial, &E);
      if (s) return s;
      if (E <= ei.energy + fp.armijo * alpha * gp) {
        accepted = true;
        break;
      }
      alpha *= 0.5;
    }
    if (!accepted) return fail(c, YASPS_E_LINESEARCH, "no admissible step after the maximum number of halvings");
    fi.alpha_min = std::min(fi.alpha_min, alpha);
    HIPCHK(c, hipMemcpyAsync(x, c->x_trial, 3 * (size_t)c->n * 8, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipEventRecord(ev[4], c->stream));
    HIPCHK(c, hipEventSynchronize(ev[4]));
    (void)hipEventElapsedTime(&ms, ev[3], ev[4]);
    fi.ms_linesearch += ms;
  }
  launch_frame_velocity(c->n, x, xs, h, v, c->stream);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (info) *info = fi;
  if (!fi.converged) return fail(c, YASPS_E_NOCONV, "Newton reached max_newton before the stop rule");
  return YASPS_OK;
}

}  // extern "C"
