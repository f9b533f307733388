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
void launch_snh_eval(const SnhArgs& a, bool exact, bool mixed, hipStream_t s);
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
// three triangle vertices are free (a kernel with a reduced projection).
constexpr int PT_TRIANGLE_FREE = 5;
void launch_contact_eval(int type, int nfree, const ContactArgs& a, bool exact, hipStream_t s);
// Device build of the dynamic part's index structures (dynindex.hip); every
// array equals the host builder's (pattern.cpp).  Input arrays are device
// memory; the static share of the full rows is the static-only FullPattern.
struct DynIndexIn {
  int n, nall, nc;
  const int32_t* type;     // [nc]
  const int32_t* idx;      // [4][nc], API order
  int nnzb_s;              // static blocks (the dynamic ones follow them in src numbering)
  const int32_t* sf_ptr;   // [n + 1] static share of each full row
  const int32_t* sf_col;
  const int32_t* sf_src;
  long long sf_nnz;
  int row_cost;            // per-row work in blocks for the XCD split
  void* arena;             // device scratch for the temporaries (may be null)
  size_t arena_bytes;
};
struct DynIndexOut {
  int err_stencil = -1, err_reason = 0;  // first invalid stencil: 1 type, 2 vertex ids, 3 no free vertex
  int gcount[32] = {};                    // stencils per group key type * 8 + nfree (or PT_TRIANGLE_FREE)
  int nnzb = 0, nent = 0, ngrad = 0;      // dynamic blocks, staged block / gradient contributions
  long long f_nnz = 0;
  int xsplit[PCG_XCDS + 1] = {};
  size_t arena_needed = 0;                // scratch the temporaries took (to size the next arena)
  // device arrays from `alloc` (owned by the caller): storage-order vertex ids
  // [4][nc], pattern rows [n + 1] / columns, slot map [nc][10] (API order),
  // staging (spos [10][nc], gpos [4][nc], cptr [nnzb + 1], gptr [n + 1]),
  // dynamic diagonal block per vertex [n], full rows (row_ptr [n + 1], col, src)
  int32_t *sidx = nullptr, *rp = nullptr, *col = nullptr, *slot = nullptr, *spos = nullptr, *gpos = nullptr,
          *cptr = nullptr, *gptr = nullptr, *ddiag = nullptr, *f_rp = nullptr, *f_col = nullptr, *f_src = nullptr;
};
// Far entries of the SpMV rows (float64): an entry below the diagonal of row r
// whose stored block is a contact block (index >= nnzb_s) in row c < r -
// far_rows (contact partners far apart in the vertex order: its second read
// would miss L2, and a miss fetches whole cache lines for 72 bytes) reads a
// transposed copy instead, kept after the stored blocks and refilled at every
// assembly (launch_far_gather).  Mesh blocks are never copied: their second
// read hits L2 often enough that a copy only adds bytes (measured).  Rewrites
// those entries' src to nnzb_total + j and returns far_src[j] = the stored
// block of copy j (nfar copies; memory from `alloc`).  0 done, -1 HIP
// failure; synchronises s.
#ifndef YASPS_FAR_ROWS
#define YASPS_FAR_ROWS 8192
#endif
constexpr int FAR_ROWS = YASPS_FAR_ROWS;
int split_far_entries(int n, const int32_t* f_rp, const int32_t* f_col, int32_t* f_src, int nnzb_s, int nnzb_total,
                      int far_rows, int32_t** far_src, int* nfar, const std::function<void*(size_t)>& alloc,
                      hipStream_t s);
// vals[9 (nnzb_total + j) ...] = transpose of stored block far_src[j]
void launch_far_gather(int nfar, const int32_t* far_src, int nnzb_total, double* vals, hipStream_t s);
// 0 built, 1 invalid contacts (err_* set), -1 HIP failure.  Synchronises s.
int build_dynamic_index(const DynIndexIn& in, DynIndexOut& out, const std::function<void*(size_t)>& alloc,
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
                        const int32_t* gptr_d, const double* stg_d, double* grad, hipStream_t s);
// Precision form: the float32 values of every full-row entry as structure of
// arrays vf[q * nnz + k] (from the stored blocks through src, as in PcgMatrix).
void launch_full_gather_f32(long long nnz, const int32_t* src, int nnzb_s, const float* vs, const float* vd,
                            float* vf, hipStream_t s);
// vals_s[row_ptr_s[v]] += shift m_v I (the diagonal block is first in its static row).
void launch_add_mass_shift(int n, const int32_t* row_ptr_s, const double* mass, double shift, double* vals_s,
                           float* vals_s32, hipStream_t s);
// Block-Jacobi inverse of static + dynamic diagonal blocks.
void launch_block_inverse(int n, const int32_t* row_ptr_s, const double* vals_s,
                          const int32_t* ddiag, const double* vals_d, double* inv,
                          uint32_t* flags, hipStream_t s);
void launch_block_inverse_f32(int n, const int32_t* row_ptr_s, const float* vals_s,
                              const int32_t* ddiag, const float* vals_d, double* inv,
                              uint32_t* flags, hipStream_t s);

// Deterministic final sums of per-workgroup partials: out[k] = sum (or min) of
// parts[off[k] .. off[k+1]).
void launch_finalize(int nseg, const int* off_host, const double* parts, const int* kind_host,
                     double* out, hipStream_t s);

// Vector helpers.
void launch_axpy_to(int n3, const double* x, double alpha, const double* p, double* y,
                    hipStream_t s);                            // y = x + alpha p
void launch_scale(int n3, const double* x, double a, double* y, hipStream_t s);  // y = a x
void launch_max_norm3(int n, const double* p, double* part, int nblk, hipStream_t s);
// per-workgroup partial sums of a . b (grid-stride, fixed order)
void launch_dot(int n3, const double* a, const double* b, double* part, int nblk, hipStream_t s);

// PCG.
struct PcgMatrix {
  int n;
  // first row of each XCD's range (xsplit[PCG_XCDS] = n), chosen on the host so
  // that the ranges hold equal work (blocks plus a per-row overhead)
  int xsplit[PCG_XCDS + 1];
  // both triangles of H_static + H_dynamic, row by row (FullPattern): per
  // entry its column and the stored upper block it is (src: static blocks
  // first, then dynamic, then the far copies; negative = transposed).
  // Float64: the values are the assembled upper blocks themselves (9
  // contiguous values each) and, for the far entries only, transposed copies
  // (split_far_entries).  Precision form: a float32 copy of every entry's
  // values as structure of arrays, v32[q * nnz + k] (measured faster for
  // 36-byte blocks than reading the stored ones).
  const int32_t* rp;
  const int32_t* col;
  const int32_t* src;
  long long nnz;
  const double* vals;  // float64: static blocks, dynamic blocks, far copies, contiguous
  const float* v32;
  const double* minv;  // (n, 9)
};
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
size_t pcg_workspace_bytes(int n);
// Size of the fixed per-GPU workspace array of the non-allocating solve
// (pcg_workspace_bytes(n) <= this for n <= 139,464 free vertices).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;
// Device address of that array on `device`, which must be the current device;
// resolved with hipGetSymbolAddress on the first call per device and kept.
hipError_t noalloc_scratch(int device, void** ptr);
// y = H x (both parts, symmetric upper storage) through the solver's SpMV kernel.
void launch_spmv(const PcgMatrix& A, const double* x, double* y, void* work, hipStream_t s);

}  // namespace yasps
