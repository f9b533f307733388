// Host-side construction of the block pattern, the slot map and the staging
// layout of the atomic-free assembly.
//
// Pattern rule (appendix "Global Hessian Compression"): collect the
// upper-triangular block coordinates of every stencil, sort them
// lexicographically by (row, col) and remove duplicates; "PositionInData" maps
// each local block of each stencil to its stored block.  Placement indices
// are 0-based with -1 for "no block" (the paper's 1-based indices with 0 as the
// pad, appendix "Index Computation").  Local pairs (a, b), a <= b, are
// enumerated row by row over the stencil's used vertices; a pair contributes
// only when both vertices are free; the static part also holds (v, v) for
// every free vertex.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace yasps {

struct PartPattern {
  int nnzb = 0;
  std::vector<int32_t> row_ptr;   // n + 1
  std::vector<int32_t> col_idx;   // nnzb
  std::vector<int32_t> slot;      // [n_stencils][10], stencil-major (API order)
};

// Builds the pattern of one part from stencils given as [width][ns] vertex (or
// row) ids, ids >= n_free having no row; slot is [ns][width (width + 1) / 2].
// `diag` adds (v, v) for every row.
void build_pattern(int n_free, const int32_t* idx_soa, int ns, bool diag, PartPattern& out, int width = 4);

// Staging layout: contributions of every slot are stored contiguously
// (cptr[slot] .. cptr[slot + 1]) in the order: optional per-vertex leading
// entry (inertia, static part only), then stencils in storage order and, within
// a stencil, local pairs in canonical order.  spos[q][s] is the staged position
// of pair q of stencil s (-1 if none).  The gradient is staged the same way per
// vertex (gptr, gpos[a][s]).
struct Staging {
  std::vector<int32_t> cptr, spos, lead_spos;  // lead_spos[v]: position of the leading block of vertex v or -1
  std::vector<int32_t> gptr, gpos, lead_gpos;  // lead_gpos[v]: position of the leading gradient entry or -1
  int nblocks = 0, ngrads = 0;
};

// `order` lists the stencils in storage order (stencil ids into idx_soa);
// slot must come from build_pattern over the same stencils (API order).  The
// leading entries are those of rows < nlead (-1: every row).
void build_staging(int n_free, const int32_t* idx_soa, int ns, const PartPattern& pat,
                   const std::vector<int32_t>& order, bool lead_block, bool lead_grad, Staging& out,
                   int width = 4, int nlead = -1);

int used_vertices(const int32_t* idx_soa, int ns, int s, int width = 4);

}  // namespace yasps
