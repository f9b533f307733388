// Internal launch interfaces between the C-ABI layer and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>

namespace yasps {

constexpr int EVAL_BLOCK = 128;   // threads per workgroup of the stencil kernels
// XCDs of the part: the SpMV-shaped kernels give each a contiguous row range.
constexpr int PCG_XCDS = 8;
constexpr int RED_BLOCK = 256;    // threads per workgroup of reductions / vector kernels

// Elastic (stable Neo-Hookean) tets.
struct SnhArgs {
  int n_free;
  const double* x;        // (n_free, 3)
  const double* x_fixed;  // (n_fixed, 3)
  int nt;
  const int32_t* idx;     // [4][nt]
  const double* dm_inv;   // [9][nt]
  const double* vol;      // [nt]
  const double* mu_lam;   // [2][nt] or null
  double mu, lam;
  double h2;
  const int32_t* spos;    // [10][nt] staged block position of each local pair, -1 = none
  const int32_t* gpos;    // [4][nt] staged gradient position of each vertex, -1 = fixed
  double* blk;            // staged 3x3 blocks (9 doubles each)
  float* blk32;           // staged blocks in float32 (precision form) or null
  double* grd;            // staged gradient 3-vectors
  double* e_part;         // one energy partial per workgroup
  uint32_t* flags;
};
// xspace: project the x-space Hessian over the free vertices instead of d2Psi/dF2.
void launch_snh_eval(const SnhArgs& a, bool exact, bool mixed, bool xspace, hipStream_t s);
// Energy only at x (line search); writes one partial per workgroup.
void launch_snh_energy(const SnhArgs& a, hipStream_t s);
// grad_theta[t] = -lambda_t . d/dx (Psi_t / theta_t)
void launch_snh_theta_adjoint(const SnhArgs& a, const double* lambda, const double* theta,
                              double* out, hipStream_t s);

// Cloth: StVK membrane triangles (3 vertices) and dihedral hinges (4).
struct MembraneArgs {
  int n_free;
  const double* x;
  const double* x_fixed;
  int nf;
  const int32_t* idx;     // [3][nf]
  const double* dm_inv;   // [4][nf] row-major 2x2 inverse rest shapes
  const double* area;     // [nf]
  double mu, lam, thick, h2;
  const int32_t* spos;    // [6][nf] staged block position per local pair (-1 = none)
  const int32_t* gpos;    // [3][nf]
  double* blk;
  float* blk32;           // float32 staged blocks (precision form) instead of blk, or null
  double* grd;
  double* e_part;
  uint32_t* flags;
};
void launch_membrane_eval(const MembraneArgs& a, bool exact, hipStream_t s);
void launch_membrane_energy(const MembraneArgs& a, hipStream_t s);

// Hinges stored grouped by number of free vertices; [begin, end) is one group.
struct HingeArgs {
  int n_free;
  const double* x;
  const double* x_fixed;
  int begin, end, nh;
  const int32_t* idx;     // [4][nh] storage order: shared edge x0, x1, wings x2, x3
  const double* rest;     // [2][nh] rest angle, stiffness
  double h2;
  const int32_t* spos;    // [10][nh]
  const int32_t* gpos;    // [4][nh]
  double* blk;
  float* blk32;
  double* grd;
  double* e_part;         // partials of this group
  uint32_t* flags;
};
void launch_hinge_eval(int nfree, const HingeArgs& a, bool exact, hipStream_t s);
void launch_hinge_energy(const HingeArgs& a, hipStream_t s);

// Inertia (dynamic) or gravity potential (static) per free vertex.
struct InertiaArgs {
  int n;
  const double* x;
  const double* x_tilde;
  const double* mass;
  int is_static;
  double g[3];
  const int32_t* spos;  // [n] staged position of m I in the static part (-1 when static)
  const int32_t* gpos;  // [n]
  double* blk;
  float* blk32;
  double* grd;
  double* e_part;
  uint32_t* flags;
};
void launch_inertia(const InertiaArgs& a, hipStream_t s);
void launch_inertia_energy(const InertiaArgs& a, hipStream_t s);

// Affine bodies: per body the inertia 1/2 (q - q~)^T (M4 (x) I3) (q - q~) (or,
// static, the gravity potential) and the orthogonality energy
// h^2 k 1/2 |A^T A - I|^2 over its four rows (a_1, a_2, a_3, t) at x rows
// nv + 4 b ...: energies, 4 gradient rows and the 10 upper 3x3 blocks.
struct BodyArgs {
  int nv, nb;             // free vertices (the bodies' rows follow them), bodies
  const double* x;        // (nv + 4 nb, 3)
  const double* x_tilde;  // (nv + 4 nb, 3); unused when static
  const double* M4;       // [nb][16]
  const double* k;        // [nb]
  double h2;
  int is_static;
  double g[3];
  const int32_t* spos;    // [10][nb] staged block positions
  const int32_t* gpos;    // [4][nb] staged gradient positions
  double* blk;
  float* blk32;
  double* grd;
  double* e_inertia;      // per workgroup
  double* e_orth;         // per workgroup
  uint32_t* flags;
};
void launch_body_eval(const BodyArgs& a, bool exact, hipStream_t s);
void launch_body_energy(const BodyArgs& a, hipStream_t s);

// Contact stencils touching affine bodies (the third part), stored grouped by
// (type, number of movable vertices).  The position of a vertex comes from the
// union of free (id < nv: x), fixed (id < nv + nfix: x_fixed) and body vertices
// (k = id - nv - nfix: A r + t from the body's rows).  Pass 1 evaluates the
// barrier over the movable positions (projected there) into position-space
// scratch; pass 2 maps it to the stencil's row list (the chain rule through
// the union) and stages the blocks and gradient rows.
struct BodyContactArgs {
  int nv, nfix;
  const double* x;
  const double* x_fixed;
  const int32_t* body_of;    // [n_body_verts]
  const double* body_rest;   // [n_body_verts][3]
  int begin, end, ns;        // group range; all stencils (stride of the SoA arrays)
  const int32_t* idx;        // [4][ns] vertex ids, storage order
  const int32_t* vpos;       // [4][ns] list position of each vertex's first row, -1 none
  const int32_t* rows;       // [8][ns] row lists, -1 padded
  const int32_t* spos;       // [36][ns] staged block positions
  const int32_t* gpos;       // [8][ns] staged gradient positions
  const double* eps;         // [ns] edge-edge mollifier thresholds in storage order, or null
  double kappa, dhat;
  int barrier;
  double* pos_blk;           // [ns][10][9] movable-pair blocks (pair order over 4)
  double* pos_grd;           // [ns][4][3]
  double* blk;
  float* blk32;
  double* grd;
  double* e_part;
  double* d_out;
  double* dmin_part;
  double* nact_part;
  uint32_t* flags;
};
void launch_body_contact_eval(int type, int nmov, const BodyContactArgs& a, bool exact, hipStream_t s);
// Line-search trial at x (already x + alpha p); x0 = the step's start for the side test.
void launch_body_contact_energy(int type, const BodyContactArgs& a, const double* x0, double* bad_part,
                                hipStream_t s);

// Contact stencils, processed in groups of equal (type, number of free vertices)
// stored contiguously.
struct ContactArgs {
  int n_free;
  const double* x;
  const double* x_fixed;
  int begin, end;        // stencil range of this group in the sorted arrays
  int nc;                // all stencils (stride of the SoA arrays)
  const int32_t* idx;    // [4][nc]
  const int32_t* spos;   // [10][nc] canonical local-pair order
  const int32_t* gpos;   // [4][nc]
  const double* eps;     // [nc] edge-edge mollifier thresholds in storage order, or null (none)
  double kappa, dhat;
  int barrier;           // 0 squared-log, 1 classic
  double* blk;
  float* blk32;          // float32 staged blocks (precision form) instead of blk, or null
  double* grd;
  double* e_part;        // per workgroup of this group (offset by the caller)
  double* d_out;         // [nc] squared distance
  double* dmin_part;     // per workgroup minimum of d
  double* nact_part;     // per workgroup count of active stencils
  uint32_t* flags;
};
// `nfree` is the number of free vertices of the group's stencils, or
// PT_TRIANGLE_FREE for point-triangle stencils whose point is fixed and whose
// three triangle vertices are free (a group and kernel of their own: the
// projection uses the triangle's uniform normal shift).
constexpr int PT_TRIANGLE_FREE = 5;
void launch_contact_eval(int type, int nfree, const ContactArgs& a, bool exact, hipStream_t s);
// Device build of the dynamic part's index structures (dynindex.hip); every
// array equals the host builder's (pattern.cpp).  Input arrays are device
// memory; the static share of the full rows is the static-only FullPattern.
struct DynIndexIn {
  int n, nall, nc;         // free vertices (ids below n have a row), all vertex ids, contacts
  int nrows;               // rows of the matrix (>= n: affine-body rows follow the free vertices)
  const int32_t* type;     // [nc]
  const int32_t* idx;      // [4][nc], API order
  const double* eps;       // [nc] edge-edge mollifier thresholds, API order, or null
  void* arena;             // device scratch for the temporaries (may be null)
  size_t arena_bytes;
  int* pin;                // pinned host scratch of PIN_INTS ints for the read-backs
};
struct DynIndexOut {
  int err_stencil = -1, err_reason = 0;  // first invalid stencil: 1 type, 2 vertex ids, 3 no free vertex
  int gcount[32] = {};                    // stencils per group key type * 8 + nfree (or PT_TRIANGLE_FREE)
  int nnzb = 0, nent = 0, ngrad = 0;      // dynamic blocks, staged block / gradient contributions
  size_t arena_needed = 0;                // scratch the temporaries took (to size the next arena)
  // device arrays from `alloc` (owned by the caller; `alloc(which, bytes)` with
  // which = the DI_* id below): storage-order vertex ids [4][nc], pattern rows
  // [n + 1] / columns, slot map [nc][10] (API order), staging (spos [10][nc],
  // gpos [4][nc], cptr [nnzb + 1], gptr [n + 1]), dynamic diagonal block per
  // vertex [n]
  int32_t *sidx = nullptr, *rp = nullptr, *col = nullptr, *slot = nullptr, *spos = nullptr, *gpos = nullptr,
          *cptr = nullptr, *gptr = nullptr, *ddiag = nullptr;
  double* seps = nullptr;  // [nc] mollifier thresholds in storage order (null without in.eps)
};
enum { DI_SIDX, DI_RP, DI_COL, DI_CPTR, DI_SLOT, DI_SPOS, DI_GPOS, DI_GPTR, DI_DDIAG, DI_EPS, DI_COUNT };
// 0 built, 1 invalid contacts (err_* set), -1 HIP failure.  Synchronises s.
int build_dynamic_index(const DynIndexIn& in, DynIndexOut& out, const std::function<void*(int, size_t)>& alloc,
                        hipStream_t s);
// Line-search trial at y = x + alpha p: energy partials, feasibility (d > 0 and
// PT/EE side kept) per workgroup.
void launch_contact_energy(int type, const ContactArgs& a, const double* x0, double* bad_part,
                           hipStream_t s);

// Segmented sums of staged contributions (atomic-free assembly).
// (ncontrib = total staged contributions, used to size the lane groups)
void launch_segsum_blocks(int nslots, long long ncontrib, const int32_t* cptr, const double* staged,
                          double* out, hipStream_t s);
void launch_segsum_blocks_f32(int nslots, long long ncontrib, const int32_t* cptr, const float* staged,
                              float* out, hipStream_t s);
void launch_segsum_grad(int n, long long ncontrib, const int32_t* gptr_s, const double* stg_s,
                        const int32_t* gptr_d, const double* stg_d, double* grad, hipStream_t s,
                        const int32_t* gptr_b = nullptr, const double* stg_b = nullptr);
// vals_s[row_ptr_s[v]] += shift m_v I (the diagonal block is first in its static row).
void launch_add_mass_shift(int n, const int32_t* row_ptr_s, const double* mass, double shift, double* vals_s,
                           float* vals_s32, hipStream_t s);
// ratio[v] = |tr(D_v)| / (3 m_v) for the assembled diagonal blocks D_v (static
// + dynamic + body-contact parts) of the first n rows.
void launch_diag_ratio(int n, const int32_t* row_ptr_s, const void* vals_s, const int32_t* ddiag, const void* vals_d,
                       const int32_t* bdiag, const void* vals_b, bool f32, const double* mass, double* ratio,
                       hipStream_t s);
// Block-Jacobi inverse of static + dynamic diagonal blocks.
// (bdiag / vals_b: the body-contact part's diagonal blocks, or null.)
void launch_block_inverse(int n, const int32_t* row_ptr_s, const double* vals_s,
                          const int32_t* ddiag, const double* vals_d, double* inv,
                          uint32_t* flags, hipStream_t s, const int32_t* bdiag = nullptr,
                          const double* vals_b = nullptr);
void launch_block_inverse_f32(int n, const int32_t* row_ptr_s, const float* vals_s,
                              const int32_t* ddiag, const float* vals_d, double* inv,
                              uint32_t* flags, hipStream_t s, const int32_t* bdiag = nullptr,
                              const float* vals_b = nullptr);

// Deterministic final sums of per-workgroup partials: out[k] = sum (or min) of
// parts[off[k] .. off[k+1]).
void launch_finalize(int nseg, const int* off_host, const double* parts, const int* kind_host,
                     double* out, hipStream_t s);

// Vector helpers.
void launch_axpy_to(int n3, const double* x, double alpha, const double* p, double* y,
                    hipStream_t s);                            // y = x + alpha p
// the same with alpha read from device memory
void launch_axpy_to_dev(int n3, const double* x, const double* alpha, const double* p, double* y, hipStream_t s);
// Newton step bound of the line search on the device: *out = min(1, 0.4 sqrt(min_d) / max_v |p_v|)
// when there are contacts and p != 0, else 1 (min_d, max |p_v| read from device memory).
void launch_step_bound(const double* min_d, const double* pmax, int contacts, double* out, hipStream_t s);
void launch_scale(int n3, const double* x, double a, double* y, hipStream_t s);  // y = a x
void launch_max_norm3(int n, const double* p, double* part, int nblk, hipStream_t s);
// per-workgroup partial sums of a . b (grid-stride, fixed order)
void launch_dot(int n3, const double* a, const double* b, double* part, int nblk, hipStream_t s);

// PCG.
// Plan of the chunked symmetric SpMV over one part of the upper-triangular
// matrix (spmvplan.hip): the stored blocks in chunks of `chunk` consecutive
// blocks; per block a packed word (its local row, the LDS entries of its two
// products), per (chunk, target row) a slot of W, per row its slots
// [hptr[j], hptr[j + 1]).
constexpr int SPMV_MAX_CHUNK = 1024;  // the packed word holds 10-bit rows and 11-bit entries
struct SpmvPart {
  int nblk = 0, nrows = 0, nchunk = 0, ntarget = 0, chunk = 0;
  int max_entries = 0;  // LDS entries (products) of the fullest chunk
  // rl: row of each compressed row (rows holding blocks), null when that is every row
  const int32_t *rl = nullptr, *col = nullptr, *m0 = nullptr, *tb = nullptr, *wslot = nullptr, *hptr = nullptr;
  const uint32_t* meta = nullptr;
  const uint16_t* tend = nullptr;
  const void* vals = nullptr;  // stored blocks [nblk][9]: double, or float in the precision form
};
// Chunk size of a part with nblk stored blocks (a power of two, 256 .. SPMV_MAX_CHUNK).
int spmv_chunk_for(long long nblk);
enum { PL_RL, PL_M0, PL_TB, PL_META, PL_TEND, PL_WSLOT, PL_HPTR, PL_COUNT };
// Builds one part's plan on the device from its row pointers [n + 1] and
// columns [nblk] (device arrays).  Plan arrays come from alloc(PL_* id,
// bytes); temporaries from the arena (or allocated and freed), pin a pinned
// host scratch of PIN_INTS ints for the read-backs, *arena_needed =
// what they took.  0 built, -1 HIP failure.  Synchronises s.
int build_spmv_plan(int n, const int32_t* rp, const int32_t* col, int nblk, const void* vals, SpmvPart& out,
                    const std::function<void*(int, size_t)>& alloc, void* arena, size_t arena_bytes,
                    size_t* arena_needed, int* pin, hipStream_t s);
constexpr int PCG_PARTS = 3;  // static, dynamic (contacts), body contacts
struct PcgMatrix {
  int n = 0;
  SpmvPart part[PCG_PARTS];  // static, dynamic, body contacts (nblk = 0 when empty)
  const double* minv = nullptr;  // (n, 9) block-Jacobi inverse
  bool f32 = false;          // stored blocks in float32 (precision form)
};
// LDS bytes the SpMV kernel may take (chunks of SPMV_MAX_CHUNK blocks).
size_t spmv_max_lds_bytes();
struct PcgState;  // device-side scalars, defined in pcg.hip
// Optional per-launch timing hook (kernel class ids as in yasps.h).  begin /
// end bracket a group of launches with stream events; kernel_events hands out
// an event pair that a single launch carries itself (hipExtLaunchKernelGGL),
// which then reads the kernel's own start and end, without the marker packets'
// dispatch gaps.
struct LaunchTimer {
  virtual void begin(int cls) = 0;
  virtual void end() = 0;
  virtual bool kernel_events(int cls, hipEvent_t* start, hipEvent_t* stop) = 0;
};
// host_state: pinned host memory of at least 128 bytes that the solver polls
// its device scalars into.  hint: in, the iteration count the caller expects
// (0 = unknown); out, the count of this solve.  It only sizes the batches of
// launches between two polls (a first batch just past the hint), never the
// arithmetic.
int pcg_solve(const PcgMatrix& A, const double* b, double* x, double rtol, int max_iter,
              bool mixed, void* work, double* rel_out, int* status_out, hipStream_t s,
              LaunchTimer* tm, void* host_state, int* hint);
// Solver workspace (state, partials, Krylov vectors, nslots SpMV slots).
size_t pcg_workspace_bytes(int n, long long nslots);
// Size of the fixed per-GPU workspace array of the non-allocating solve.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
// Device address of that array on `device`, which must be the current device;
// resolved with hipGetSymbolAddress on the first call per device and kept.
hipError_t noalloc_scratch(int device, void** ptr);
// y = H x (both parts, symmetric upper storage) through the solver's SpMV kernel.
void launch_spmv(const PcgMatrix& A, const double* x, double* y, void* work, hipStream_t s, LaunchTimer* tm);

// Collision surface and positions of the proximity search / CCD (collision.hip).
struct CdSurface {
  int np, ne, nt;          // points, edges, triangles
  const int32_t* points;   // [np] vertex ids
  const int32_t* edges;    // [2][ne]
  const int32_t* tris;     // [3][nt]
  const double* len2;      // [ne] squared rest lengths (EE mollifier thresholds) or null
  double cell;             // grid cell size
};
struct CdPositions {
  int nv;                  // free vertices (ids below nv are rows of x)
  int nfix;                // fixed vertices (ids nv .. nv + nfix); body vertices follow
  const double* x;         // rows of degrees of freedom: free positions, then a_1, a_2, a_3, t per body
  const double* xf;        // fixed positions
  const int32_t* body_of;  // [body vertices] body of each, or null without bodies
  const double* body_rest; // [body vertices][3] rest positions r (p = A r + t)
  const double* p;         // motion of the rows (CCD: swept boxes over x + t p) or null
  double t;
};
struct CdOutput {
  int n = 0;               // stencils found
  int32_t* type = nullptr; // [n]
  int32_t* idx = nullptr;  // [4][n] (stride n)
  double* eps = nullptr;   // [n] mollifier thresholds (0 for the non-EE stencils)
};
// Grow-only buffers of the collision module: the registrations of the
// triangles and of the edges (cell and primitive of every entry, first entry
// of every cell), and the detected stencils.
enum { CD_REG_T, CD_REG_T_V, CD_REG_T_C, CD_REG_E, CD_REG_E_V, CD_REG_E_C, CD_TYPE, CD_IDX, CD_EPS, CD_COUNT };
using CdAlloc = std::function<void*(int, size_t)>;
// Contact stencils at X (squared distance below dhat), in the fixed order
// (point-triangle pairs by (point, triangle), then edge-edge pairs by (edge,
// edge)).  0 ok, -1 HIP failure, -2 a primitive's box over too many grid cells
// (a non-finite position or a cell size far below the motion).  Synchronises s.
int cd_detect(const CdSurface& S, const CdPositions& X, double dhat, const CdAlloc& alloc, void* arena,
              size_t arena_bytes, size_t* arena_needed, int* pin, hipStream_t s, CdOutput& out);
// Barrier energy of the stencils found at X (the same pairs as cd_detect).
int cd_energy(const CdSurface& S, const CdPositions& X, double dhat, double kappa, int classic, const CdAlloc& alloc,
              void* arena, size_t arena_bytes, size_t* arena_needed, int* pin, hipStream_t s, double* e_out);
// Largest conservative step t <= t_max along X.x + t X.p (additive CCD over the
// candidate pairs of the swept boxes).
int cd_ccd(const CdSurface& S, const CdPositions& X, double dhat, double t_max, double s_ccd, const CdAlloc& alloc,
           void* arena, size_t arena_bytes, size_t* arena_needed, int* pin, hipStream_t s, double* t_out);
// Time stepping: x_tilde = x + h v + h^2 g over the n rows (gravity on the free
// rows and the bodies' t rows) and v = (x - x_start) / h.
void launch_frame_tilde(int nv, int n, const double* x, const double* v, double h, const double g[3], double* xt,
                        hipStream_t s);
void launch_frame_velocity(int n, const double* x, const double* xs, double h, double* v, hipStream_t s);

}  // namespace yasps
