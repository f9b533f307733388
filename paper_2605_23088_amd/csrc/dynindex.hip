// Device build of the dynamic (contact) part's index structures: validation,
// storage order, block pattern and slot map, and staging layout (the SpMV plan
// of the part is built from the pattern afterwards, spmvplan.hip).
//
// The rules are those of the host builder (pattern.h / pattern.cpp, appendix
// "Global Hessian Compression"): the block pattern is the sorted, deduplicated
// set of upper block coordinates of every free pair of every stencil; the
// stencils are stored grouped by (type, number of free vertices), stably; the
// contributions of a block are staged contiguously in storage order of their
// stencils and, within a stencil, in canonical pair order.  Sorting is done by
// stable LSD radix sorts (rocPRIM), so every array equals the host builder's,
// element for element.  The paper rebuilds only this part when the contacts
// change (section "Implementation", static / dynamic split).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "devsort.h"
#include "kernels.h"

namespace yasps {

using namespace devsort;

namespace {

YDEV int verts_of(int t) { return t == 3 ? 2 : (t == 2 ? 3 : 4); }

// Per stencil (API order): the first failing check (1 unknown type, 2 bad or
// repeated vertex ids, 3 no free vertex) folded into err = min((s << 2) | reason),
// else the group key type * 8 + (free count, or PT_TRIANGLE_FREE).
YDEV void classify_one(int s, int nc, int n, int nall, const int32_t* __restrict__ type,
                       const int32_t* __restrict__ idx, uint32_t* __restrict__ gkey, int* err, int* hist) {
  if (s >= nc) return;
  const int t = type[s];
  int reason = 0, nf = 0;
  if (t < 0 || t > 3) {
    reason = 1;
  } else {
    const int nv = verts_of(t);
    int v[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) v[a] = idx[(size_t)a * nc + s];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (a < nv) {
        if (v[a] < 0 || v[a] >= nall) reason = 2;
#pragma unroll
        for (int b = 0; b < a; ++b)
          if (v[b] == v[a]) reason = 2;
        nf += (v[a] >= 0 && v[a] < n) ? 1 : 0;
      } else if (v[a] != -1) {
        reason = 2;
      }
    }
    if (!reason && nf == 0) reason = 3;
  }
  if (reason) {
    atomicMin(err, (s << 2) | reason);
    gkey[s] = 31;
    return;
  }
  const bool pt_fixed_point = t == 0 && nf == 3 && idx[s] >= n;
  const uint32_t key = (uint32_t)(t * 8 + (pt_fixed_point ? PT_TRIANGLE_FREE : nf));
  gkey[s] = key;
  atomicAdd(&hist[key], 1);
}

__global__ __launch_bounds__(DI_BLOCK) void classify_kernel(int nc, int n, int nall, const int32_t* __restrict__ type,
                                                            const int32_t* __restrict__ idx,
                                                            uint32_t* __restrict__ gkey, int* err, int* gcount) {
  // group counts: a workgroup histogram in LDS, one global add per nonzero bin
  __shared__ int hist[32];
  if (threadIdx.x < 32) hist[threadIdx.x] = 0;
  __syncthreads();
  const int s = blockIdx.x * DI_BLOCK + threadIdx.x;
  classify_one(s, nc, n, nall, type, idx, gkey, err, hist);
  __syncthreads();
  if (threadIdx.x < 32 && hist[threadIdx.x]) atomicAdd(&gcount[threadIdx.x], hist[threadIdx.x]);
}

// Per stencil in storage order j (s = order[j]): its vertex ids in storage
// order, one block entry per canonical pair q (key (r << 32) | c of a free pair,
// else the pad key, which sorts last) and one gradient entry per used vertex
// (its id if free, else the pad n).
__global__ void entries_kernel(int nc, int n, const int32_t* __restrict__ idx, const int32_t* __restrict__ order,
                               uint64_t pad, int32_t* __restrict__ sidx, uint64_t* __restrict__ bkey,
                               int32_t* __restrict__ bval, uint32_t* __restrict__ gkey, int32_t* __restrict__ gval,
                               int* counts, const double* __restrict__ eps, double* __restrict__ seps) {
  const int j = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (j >= nc) return;
  const int s = order[j];
  if (eps) seps[j] = eps[s];
  int v[4];
  int used = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    v[a] = idx[(size_t)a * nc + s];
    sidx[(size_t)a * nc + j] = v[a];
    used += v[a] >= 0 ? 1 : 0;
  }
  int q = 0, nb = 0, ng = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) {
      if (a < used && b < used) {
        const bool fr = v[a] < n && v[b] < n;
        const uint64_t r = (uint64_t)min(v[a], v[b]), c = (uint64_t)max(v[a], v[b]);
        bkey[(size_t)j * 10 + q] = fr ? ((r << 32) | c) : pad;
        nb += fr ? 1 : 0;
        ++q;
      }
    }
  for (; q < 10; ++q) bkey[(size_t)j * 10 + q] = pad;
#pragma unroll
  for (int k = 0; k < 10; ++k) bval[(size_t)j * 10 + k] = j * 10 + k;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const bool fr = v[a] >= 0 && v[a] < n;
    gkey[(size_t)j * 4 + a] = fr ? (uint32_t)v[a] : (uint32_t)n;
    gval[(size_t)j * 4 + a] = j * 4 + a;
    ng += fr ? 1 : 0;
  }
  atomicAdd(&counts[0], nb);
  atomicAdd(&counts[1], ng);
}

// first[i] = 1 where sorted block entry i opens a new block
__global__ void first_kernel(int ne, const uint64_t* __restrict__ key, int32_t* __restrict__ first) {
  const int i = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i >= ne) return;
  first[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

// Block entries (sorted, i < ne; blk = inclusive count of block starts):
// staged positions, block columns, contribution starts, slot map (API order),
// per-row block counts, dynamic diagonal positions and the off-diagonal count.
__global__ void blocks_kernel(int ne, int nc, const uint64_t* __restrict__ key, const int32_t* __restrict__ val,
                              const int32_t* __restrict__ blk, const int32_t* __restrict__ first,
                              const int32_t* __restrict__ order, int32_t* __restrict__ spos,
                              int32_t* __restrict__ col, int32_t* __restrict__ cptr, int32_t* __restrict__ slot,
                              int32_t* __restrict__ rowcnt, int32_t* __restrict__ ddiag, int* offdiag) {
  const int i = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i >= ne) return;
  const int jq = val[i], j = jq / 10, q = jq - 10 * (jq / 10);
  const int b = blk[i] - 1;
  spos[(size_t)q * nc + j] = i;
  slot[(size_t)order[j] * 10 + q] = b;
  if (first[i]) {
    const int r = (int)(key[i] >> 32), c = (int)(key[i] & 0xffffffffu);
    col[b] = c;
    cptr[b] = i;
    atomicAdd(&rowcnt[r], 1);
    if (r == c)
      ddiag[r] = b;
    else
      atomicAdd(offdiag, 1);
  }
}

// Gradient entries (sorted by vertex, i < ng): staged positions, per-vertex counts.
__global__ void grads_kernel(int ng, int nc, const int32_t* __restrict__ val, int32_t* __restrict__ gpos) {
  const int i = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i >= ng) return;
  const int ja = val[i], j = ja / 4, a = ja - 4 * (ja / 4);
  gpos[(size_t)a * nc + j] = i;
}

// gptr[v] = first sorted gradient entry of vertex v (v = 0 .. n; entries of
// vertex v are [gptr[v], gptr[v + 1]))
__global__ void gptr_kernel(int n, int ng, const uint32_t* __restrict__ key, int32_t* __restrict__ gptr) {
  const int v = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (v > n) return;
  int lo = 0, hi = ng;
  while (lo < hi) {
    const int mid = (lo + hi) / 2;
    if (key[mid] < (uint32_t)v)
      lo = mid + 1;
    else
      hi = mid;
  }
  gptr[v] = lo;
}

__global__ void fill_i32_kernel(long long m, int32_t v, int32_t* __restrict__ p) {
  const long long i = (long long)blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i < m) p[i] = v;
}

__global__ void iota_kernel(int m, int32_t* __restrict__ p) {
  const int i = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i < m) p[i] = i;
}

}  // namespace

#define DI_CHECK(expr)                       \
  do {                                       \
    const hipError_t e_ = (expr);            \
    if (e_ != hipSuccess) return -1;         \
  } while (0)

int build_dynamic_index(const DynIndexIn& in, DynIndexOut& out, const std::function<void*(int, size_t)>& alloc,
                        hipStream_t s) {
  const int n = in.n, nc = in.nc;
  Temp tmp;
  tmp.arena = static_cast<char*>(in.arena);
  tmp.cap = in.arena_bytes;
  out = DynIndexOut{};
  struct Need {  // reports the arena size the build needed, on every return path
    Temp& t;
    DynIndexOut& o;
    ~Need() { o.arena_needed = t.used; }
  } need{tmp, out};
  // small device scalars: err, counts[2] (block / gradient entries), offdiag, gcount[32]
  int* scal = tmp.get<int>(48);
  DI_CHECK(tmp.err);
  int* err = scal;
  int* counts = scal + 1;
  int* offdiag = scal + 3;
  int* gcount = scal + 4;
  const int init[4] = {0x7fffffff, 0, 0, 0};
  DI_CHECK(hipMemsetAsync(scal, 0, 48 * sizeof(int), s));
  DI_CHECK(hipMemcpyAsync(scal, init, sizeof(init), hipMemcpyHostToDevice, s));

  // 1. validation, group keys, storage order (stable by group key)
  uint32_t* gk = tmp.get<uint32_t>(nc);
  uint32_t* gk_sorted = tmp.get<uint32_t>(nc);
  int32_t* iota = tmp.get<int32_t>(nc);
  int32_t* order = tmp.get<int32_t>(nc);
  DI_CHECK(tmp.err);
  if (nc) {
    hipLaunchKernelGGL(classify_kernel, dim3(grid_of(nc)), dim3(DI_BLOCK), 0, s, nc, n, in.nall, in.type, in.idx,
                       gk, err, gcount);
    hipLaunchKernelGGL(iota_kernel, dim3(grid_of(nc)), dim3(DI_BLOCK), 0, s, nc, iota);
    DI_CHECK(sort_pairs(tmp, gk, gk_sorted, iota, order, nc, 5, s));
  }
  int head[36];
  DI_CHECK(hipMemcpyAsync(head, scal, sizeof(head), hipMemcpyDeviceToHost, s));
  DI_CHECK(hipStreamSynchronize(s));
  if (head[0] != 0x7fffffff) {
    out.err_stencil = head[0] >> 2;
    out.err_reason = head[0] & 3;
    return 1;
  }
  std::copy(head + 4, head + 36, out.gcount);

  // 2. block and gradient entries in storage order; stable sorts by block / vertex
  const long long nbe = 10ll * nc, nge = 4ll * nc;
  const int nbits = bits_for(n);
  const uint64_t bpad = (uint64_t)n << 32;  // above every (r << 32) | c with r, c < n
  uint64_t* bkey = tmp.get<uint64_t>(nbe);
  uint64_t* bkey_s = tmp.get<uint64_t>(nbe);
  int32_t* bval = tmp.get<int32_t>(nbe);
  int32_t* bval_s = tmp.get<int32_t>(nbe);
  uint32_t* gkey = tmp.get<uint32_t>(nge);
  uint32_t* gkey_s = tmp.get<uint32_t>(nge);
  int32_t* gval = tmp.get<int32_t>(nge);
  int32_t* gval_s = tmp.get<int32_t>(nge);
  int32_t* sidx = static_cast<int32_t*>(alloc(DI_SIDX, sizeof(int32_t) * std::max<long long>(nge, 1)));
  double* seps = in.eps ? static_cast<double*>(alloc(DI_EPS, sizeof(double) * std::max(nc, 1))) : nullptr;
  DI_CHECK(tmp.err);
  if (!sidx || (in.eps && !seps)) return -1;
  if (nc) {
    hipLaunchKernelGGL(entries_kernel, dim3(grid_of(nc)), dim3(DI_BLOCK), 0, s, nc, n, in.idx, order, bpad, sidx,
                       bkey, bval, gkey, gval, counts, in.eps, seps);
    DI_CHECK(sort_pairs(tmp, bkey, bkey_s, bval, bval_s, nbe, 32 + nbits, s));
    DI_CHECK(sort_pairs(tmp, gkey, gkey_s, gval, gval_s, nge, nbits, s));
  }
  int cnt[2];
  DI_CHECK(hipMemcpyAsync(cnt, counts, sizeof(cnt), hipMemcpyDeviceToHost, s));
  DI_CHECK(hipStreamSynchronize(s));
  const int ne = cnt[0], ng = cnt[1];

  // 3. blocks: starts, indices, pattern, slot map, staging
  int32_t* first = tmp.get<int32_t>(ne);
  int32_t* blk = tmp.get<int32_t>(ne);
  DI_CHECK(tmp.err);
  int nnzb = 0;
  if (ne) {
    hipLaunchKernelGGL(first_kernel, dim3(grid_of(ne)), dim3(DI_BLOCK), 0, s, ne, bkey_s, first);
    DI_CHECK(inclusive(tmp, first, blk, ne, s));
    DI_CHECK(hipMemcpyAsync(&nnzb, blk + ne - 1, sizeof(int), hipMemcpyDeviceToHost, s));
    DI_CHECK(hipStreamSynchronize(s));
  }
  auto ialloc = [&](int which, long long m) {
    return static_cast<int32_t*>(alloc(which, sizeof(int32_t) * std::max<long long>(m, 1)));
  };
  const int nr = std::max(in.nrows, n);  // row arrays span every row (the rows past n stay empty)
  out.rp = ialloc(DI_RP, nr + 1);
  out.col = ialloc(DI_COL, nnzb);
  out.cptr = ialloc(DI_CPTR, nnzb + 1);
  out.slot = ialloc(DI_SLOT, 10ll * nc);
  out.spos = ialloc(DI_SPOS, 10ll * nc);
  out.gpos = ialloc(DI_GPOS, 4ll * nc);
  out.gptr = ialloc(DI_GPTR, nr + 1);
  out.ddiag = ialloc(DI_DDIAG, nr);
  out.sidx = sidx;
  out.seps = seps;
  if (!out.rp || !out.col || !out.cptr || !out.slot || !out.spos || !out.gpos || !out.gptr || !out.ddiag) return -1;
  int32_t* rowcnt = tmp.get<int32_t>(nr);
  DI_CHECK(tmp.err);
  DI_CHECK(hipMemsetAsync(rowcnt, 0, sizeof(int32_t) * std::max(nr, 1), s));
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_of(10ll * nc)), dim3(DI_BLOCK), 0, s, 10ll * nc, -1, out.slot);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_of(10ll * nc)), dim3(DI_BLOCK), 0, s, 10ll * nc, -1, out.spos);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_of(4ll * nc)), dim3(DI_BLOCK), 0, s, 4ll * nc, -1, out.gpos);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_of(nr)), dim3(DI_BLOCK), 0, s, (long long)nr, -1, out.ddiag);
  if (ne)
    hipLaunchKernelGGL(blocks_kernel, dim3(grid_of(ne)), dim3(DI_BLOCK), 0, s, ne, nc, bkey_s, bval_s, blk, first,
                       order, out.spos, out.col, out.cptr, out.slot, rowcnt, out.ddiag, offdiag);
  DI_CHECK(hipMemcpyAsync(out.cptr + nnzb, &ne, sizeof(int), hipMemcpyHostToDevice, s));
  DI_CHECK(prefix(tmp, rowcnt, out.rp, nr, s));
  if (ng) hipLaunchKernelGGL(grads_kernel, dim3(grid_of(ng)), dim3(DI_BLOCK), 0, s, ng, nc, gval_s, out.gpos);
  hipLaunchKernelGGL(gptr_kernel, dim3(grid_of(nr + 1)), dim3(DI_BLOCK), 0, s, nr, ng, gkey_s, out.gptr);

  DI_CHECK(hipGetLastError());
  DI_CHECK(hipStreamSynchronize(s));  // the temporaries go out of scope
  out.nnzb = nnzb;
  out.nent = ne;
  out.ngrad = ng;
  return 0;
}

}  // namespace yasps
