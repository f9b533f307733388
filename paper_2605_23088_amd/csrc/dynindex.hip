// Device build of the dynamic (contact) part's index structures: validation,
// storage order, block pattern and slot map, and staging layout (the SpMV plan
// of the part is built from the pattern afterwards, spmvplan.hip).
//
// The rules are those of the host builder (pattern.h / pattern.cpp, appendix
// "Global Hessian Compression"): the block pattern is the sorted, deduplicated
// set of upper block coordinates of every free pair of every stencil; the
// stencils are stored grouped by (type, number of free vertices), stably; the
// contributions of a block are staged contiguously in storage order of their
// stencils and, within a stencil, in canonical pair order.  The storage order
// comes from a stable counting sort by group key; the block entries (one per
// free pair, written compacted) are ordered by a stable LSD radix sort
// (rocPRIM) over only the key bits in use; the gradient entries are the
// diagonal blocks' entries in that order.  Every array equals the host
// builder's, element for element.  One host round trip
// (the group counts, which size everything after them) precedes the final
// synchronisation.  The paper rebuilds only this part when the contacts
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
                                                            uint32_t* __restrict__ gkey, int* err, int* gcount,
                                                            int* __restrict__ blkhist) {
  // group counts: a workgroup histogram in LDS, one global add per nonzero bin,
  // and the workgroup's count of every key (key-major) for the stable scatter
  __shared__ int hist[32];
  if (threadIdx.x < 32) hist[threadIdx.x] = 0;
  __syncthreads();
  const int s = blockIdx.x * DI_BLOCK + threadIdx.x;
  classify_one(s, nc, n, nall, type, idx, gkey, err, hist);
  __syncthreads();
  if (threadIdx.x < 32) {
    blkhist[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = hist[threadIdx.x];
    if (hist[threadIdx.x]) atomicAdd(&gcount[threadIdx.x], hist[threadIdx.x]);
  }
}

// Stable counting sort by group key (keys < 32): base = exclusive prefix of the
// key-major workgroup counts; a stencil's rank among the equal keys of its
// workgroup comes from wavefront ballots (lanes with the same key below it)
// plus the counts of the same key in the workgroup's earlier wavefronts.
__global__ __launch_bounds__(DI_BLOCK) void group_scatter_kernel(int nc, const uint32_t* __restrict__ gkey,
                                                                 const int32_t* __restrict__ base,
                                                                 int32_t* __restrict__ order) {
  constexpr int NW = DI_BLOCK / 64;
  __shared__ int cnt[NW][32];
  for (int t = threadIdx.x; t < NW * 32; t += DI_BLOCK) cnt[t / 32][t % 32] = 0;
  __syncthreads();
  const int s = blockIdx.x * DI_BLOCK + threadIdx.x;
  const bool in = s < nc;
  const uint32_t k = in ? gkey[s] : 0u;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t same = __ballot(in);
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    const uint64_t ones = __ballot(in && ((k >> b) & 1u));
    same &= ((k >> b) & 1u) ? ones : ~ones;
  }
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int rank = __popcll(same & below);
  if (in && rank == 0) cnt[w][k] = __popcll(same);
  __syncthreads();
  if (!in) return;
  int off = base[(size_t)k * gridDim.x + blockIdx.x] + rank;
  for (int q = 0; q < w; ++q) off += cnt[q][k];
  order[off] = s;
}

// Per stencil in storage order j (s = order[j]): its vertex ids and mollifier
// threshold in storage order, and -1 in the staging positions and slot-map
// entries of its pairs and vertices that are not free (the free ones are
// written by blocks_kernel).
__global__ void stencil_kernel(int nc, int n, const int32_t* __restrict__ idx, const int32_t* __restrict__ order,
                               int32_t* __restrict__ sidx, const double* __restrict__ eps,
                               double* __restrict__ seps, int32_t* __restrict__ spos, int32_t* __restrict__ slot,
                               int32_t* __restrict__ gpos) {
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
  int q = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) {
      const bool pair = a < used && b < used;
      const bool fr = pair && v[a] < n && v[b] < n;
      if (pair) {
        if (!fr) {
          spos[(size_t)q * nc + j] = -1;
          slot[(size_t)s * 10 + q] = -1;
        }
        ++q;
      }
    }
  for (int r = q; r < 10; ++r) {
    spos[(size_t)r * nc + j] = -1;
    slot[(size_t)s * 10 + r] = -1;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
    if (!(v[a] >= 0 && v[a] < n)) gpos[(size_t)a * nc + j] = -1;
}

// The groups in storage order: first stencil, free vertices, vertices and
// first block entry of each (every stencil of a group has the same number of
// free vertices, hence nf (nf + 1) / 2 block entries).
struct GroupTable {
  int ng;
  int begin[32], nf[32], nv[32];
  int ebase[33];
};

YDEV int group_of(const GroupTable& T, long long e, const int* base) {
  int g = 0;
  for (int q = 1; q < T.ng; ++q) g = e >= base[q] ? q : g;
  return g;
}

// One block entry per free pair (e < ne, in storage order of the stencils and
// canonical pair order within one): key (r << bits) | c, value j * 10 + q
// (q = the pair's index among the stencil's used pairs).
__global__ void bentries_kernel(int ne, int nc, int n, int bits, GroupTable T, const int32_t* __restrict__ sidx,
                                uint64_t* __restrict__ bkey, int32_t* __restrict__ bval) {
  const int e = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (e >= ne) return;
  const int g = group_of(T, e, T.ebase);
  const int nf = T.nf[g], P = nf * (nf + 1) / 2;
  const int local = e - T.ebase[g], jl = local / P, t = local - jl * P;
  const int j = T.begin[g] + jl;
  int v[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) v[a] = sidx[(size_t)a * nc + j];
  int q = 0, f = 0, qs = 0, rs = 0, cs = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) {
      const bool pair = v[a] >= 0 && v[b] >= 0;
      const bool fr = pair && v[a] < n && v[b] < n;
      if (fr && f == t) {
        qs = q;
        rs = min(v[a], v[b]);
        cs = max(v[a], v[b]);
      }
      f += fr ? 1 : 0;
      q += pair ? 1 : 0;
    }
  bkey[e] = ((uint64_t)rs << bits) | (uint64_t)cs;
  bval[e] = j * 10 + qs;
}

// first[i] = 1 where sorted block entry i opens a new block; diag[i] = 1 on a
// diagonal block's entries.  A stencil stages one diagonal entry per free
// vertex, so the diagonal entries in sorted order are the gradient entries in
// the gradient staging order (by vertex, then storage order of the stencils).
__global__ void first_kernel(int ne, int bits, const uint64_t* __restrict__ key, int32_t* __restrict__ first,
                             int32_t* __restrict__ diag) {
  const int i = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i >= ne) return;
  const uint64_t k = key[i];
  first[i] = (i == 0 || k != key[i - 1]) ? 1 : 0;
  diag[i] = (k >> bits) == (k & ((1ull << bits) - 1)) ? 1 : 0;
}

// Block entries (sorted, i < ne; blk = inclusive count of block starts, dpos =
// exclusive count of diagonal entries): staged positions, block columns,
// contribution starts, slot map (API order), per-row block counts, dynamic
// diagonal positions, the off-diagonal count and the gradient staging
// positions; the last thread closes cptr (cptr[nnzb] = ne).
__global__ void blocks_kernel(int ne, int nc, int bits, GroupTable T, const uint64_t* __restrict__ key,
                              const int32_t* __restrict__ val, const int32_t* __restrict__ blk,
                              const int32_t* __restrict__ first, const int32_t* __restrict__ diag,
                              const int32_t* __restrict__ dpos, const int32_t* __restrict__ order,
                              int32_t* __restrict__ spos, int32_t* __restrict__ col, int32_t* __restrict__ cptr,
                              int32_t* __restrict__ slot, int32_t* __restrict__ rowcnt, int32_t* __restrict__ ddiag,
                              int32_t* __restrict__ gpos, int* offdiag) {
  const int i = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i >= ne) return;
  const int jq = val[i], j = jq / 10, q = jq - 10 * (jq / 10);
  const int b = blk[i] - 1;
  spos[(size_t)q * nc + j] = i;
  slot[(size_t)order[j] * 10 + q] = b;
  if (i == ne - 1) cptr[b + 1] = ne;
  if (diag[i]) {
    // q = the diagonal pair (a, a) among the stencil's nv used vertices:
    // q = a nv - a (a - 1) / 2
    const int nv = T.nv[group_of(T, j, T.begin)];
    int a = 0;
#pragma unroll
    for (int t = 1; t < 4; ++t) a = q == t * nv - (t * (t - 1)) / 2 ? t : a;
    gpos[(size_t)a * nc + j] = dpos[i];
  }
  if (first[i]) {
    const uint64_t k = key[i];
    const int r = (int)(k >> bits), c = (int)(k & ((1ull << bits) - 1));
    col[b] = c;
    cptr[b] = i;
    atomicAdd(&rowcnt[r], 1);
    if (r == c)
      ddiag[r] = b;
    else
      atomicAdd(offdiag, 1);
  }
}

// gradient entries of every row: the contributions of its dynamic diagonal block
__global__ void gcount_kernel(int nr, const int32_t* __restrict__ ddiag, const int32_t* __restrict__ cptr,
                              int32_t* __restrict__ gcnt) {
  const int v = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (v >= nr) return;
  const int b = ddiag[v];
  gcnt[v] = b >= 0 ? cptr[b + 1] - cptr[b] : 0;
}

__global__ void fill_i32_kernel(long long m, int32_t v, int32_t* __restrict__ p) {
  const long long i = (long long)blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i < m) p[i] = v;
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
  // small device scalars: err, nnzb, offdiag, gcount[32]
  int* scal = tmp.get<int>(48);
  DI_CHECK(tmp.err);
  int* err = scal;
  int* offdiag = scal + 3;
  int* gcount = scal + 4;
  const int init[4] = {0x7fffffff, 0, 0, 0};
  DI_CHECK(hipMemsetAsync(scal, 0, 48 * sizeof(int), s));
  DI_CHECK(hipMemcpyAsync(scal, init, sizeof(init), hipMemcpyHostToDevice, s));

  // 1. validation, group keys, storage order (a stable counting sort by group key)
  const int nwg = grid_of(nc);
  uint32_t* gk = tmp.get<uint32_t>(nc);
  int32_t* blkhist = tmp.get<int32_t>(32ll * nwg);
  int32_t* blkbase = tmp.get<int32_t>(32ll * nwg + 1);
  int32_t* order = tmp.get<int32_t>(nc);
  DI_CHECK(tmp.err);
  if (nc) {
    hipLaunchKernelGGL(classify_kernel, dim3(nwg), dim3(DI_BLOCK), 0, s, nc, n, in.nall, in.type, in.idx, gk, err,
                       gcount, blkhist);
    DI_CHECK(prefix(tmp, blkhist, blkbase, 32ll * nwg, s));
    hipLaunchKernelGGL(group_scatter_kernel, dim3(nwg), dim3(DI_BLOCK), 0, s, nc, gk, blkbase, order);
  }
  int* head = in.pin;  // err, -, -, offdiag, gcount[32]
  DI_CHECK(hipMemcpyAsync(head, scal, 36 * sizeof(int), hipMemcpyDeviceToHost, s));
  DI_CHECK(hipStreamSynchronize(s));
  if (head[0] != 0x7fffffff) {
    out.err_stencil = head[0] >> 2;
    out.err_reason = head[0] & 3;
    return 1;
  }
  std::copy(head + 4, head + 36, out.gcount);
  GroupTable T{};
  long long ne = 0, ng = 0;
  for (int key = 0, j = 0; key < 32; ++key) {
    const int cnt = out.gcount[key];
    if (!cnt) continue;
    const int nf = key % 8 == PT_TRIANGLE_FREE ? 3 : key % 8;
    const int type = key / 8;
    T.begin[T.ng] = j;
    T.nf[T.ng] = nf;
    T.nv[T.ng] = type == 3 ? 2 : (type == 2 ? 3 : 4);
    T.ebase[T.ng] = (int)ne;
    ++T.ng;
    j += cnt;
    ne += (long long)cnt * (nf * (nf + 1) / 2);
    ng += (long long)cnt * nf;
  }
  T.ebase[T.ng] = (int)ne;

  // 2. the output arrays (slot-map and staging entries of pairs or vertices
  //    that are not free are -1), storage-order stencils
  auto ialloc = [&](int which, long long m) {
    return static_cast<int32_t*>(alloc(which, sizeof(int32_t) * std::max<long long>(m, 1)));
  };
  const int nr = std::max(in.nrows, n);  // row arrays span every row (the rows past n stay empty)
  out.sidx = ialloc(DI_SIDX, 4ll * nc);
  out.seps = in.eps ? static_cast<double*>(alloc(DI_EPS, sizeof(double) * std::max(nc, 1))) : nullptr;
  out.rp = ialloc(DI_RP, nr + 1);
  out.col = ialloc(DI_COL, ne);           // nnzb <= ne
  out.cptr = ialloc(DI_CPTR, ne + 1);
  out.slot = ialloc(DI_SLOT, 10ll * nc);
  out.spos = ialloc(DI_SPOS, 10ll * nc);
  out.gpos = ialloc(DI_GPOS, 4ll * nc);
  out.gptr = ialloc(DI_GPTR, nr + 1);
  out.ddiag = ialloc(DI_DDIAG, nr);
  if (!out.sidx || (in.eps && !out.seps) || !out.rp || !out.col || !out.cptr || !out.slot || !out.spos ||
      !out.gpos || !out.gptr || !out.ddiag)
    return -1;
  if (nc)
    hipLaunchKernelGGL(stencil_kernel, dim3(nwg), dim3(DI_BLOCK), 0, s, nc, n, in.idx, order, out.sidx, in.eps,
                       out.seps, out.spos, out.slot, out.gpos);

  // 3. block entries of the free pairs in storage order, stably sorted by
  //    block (r, c); the gradient entries are the diagonal blocks' entries
  const int nbits = bits_for(n);
  uint64_t* bkey = tmp.get<uint64_t>(ne);
  uint64_t* bkey_s = tmp.get<uint64_t>(ne);
  int32_t* bval = tmp.get<int32_t>(ne);
  int32_t* bval_s = tmp.get<int32_t>(ne);
  int32_t* first = tmp.get<int32_t>(ne);
  int32_t* blk = tmp.get<int32_t>(ne);
  int32_t* diag = tmp.get<int32_t>(ne);
  int32_t* dpos = tmp.get<int32_t>(ne + 1);
  int32_t* rowcnt = tmp.get<int32_t>(nr);
  int32_t* gcnt = tmp.get<int32_t>(nr);
  DI_CHECK(tmp.err);
  if (ne) {
    hipLaunchKernelGGL(bentries_kernel, dim3(grid_of(ne)), dim3(DI_BLOCK), 0, s, (int)ne, nc, n, nbits, T,
                       out.sidx, bkey, bval);
    DI_CHECK(sort_pairs(tmp, bkey, bkey_s, bval, bval_s, ne, 2 * nbits, s));
  }

  // 4. blocks: starts, indices, pattern, slot map, staging
  DI_CHECK(hipMemsetAsync(rowcnt, 0, sizeof(int32_t) * std::max(nr, 1), s));
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_of(nr)), dim3(DI_BLOCK), 0, s, (long long)nr, -1, out.ddiag);
  if (ne) {
    hipLaunchKernelGGL(first_kernel, dim3(grid_of(ne)), dim3(DI_BLOCK), 0, s, (int)ne, nbits, bkey_s, first, diag);
    DI_CHECK(inclusive(tmp, first, blk, ne, s));
    DI_CHECK(prefix(tmp, diag, dpos, ne, s));
    hipLaunchKernelGGL(blocks_kernel, dim3(grid_of(ne)), dim3(DI_BLOCK), 0, s, (int)ne, nc, nbits, T, bkey_s,
                       bval_s, blk, first, diag, dpos, order, out.spos, out.col, out.cptr, out.slot, rowcnt,
                       out.ddiag, out.gpos, offdiag);
  } else {
    DI_CHECK(hipMemsetAsync(out.cptr, 0, sizeof(int32_t), s));
  }
  DI_CHECK(prefix(tmp, rowcnt, out.rp, nr, s));
  hipLaunchKernelGGL(gcount_kernel, dim3(grid_of(nr)), dim3(DI_BLOCK), 0, s, nr, out.ddiag, out.cptr, gcnt);
  DI_CHECK(prefix(tmp, gcnt, out.gptr, nr, s));

  in.pin[40] = 0;
  if (ne) DI_CHECK(hipMemcpyAsync(in.pin + 40, blk + ne - 1, sizeof(int), hipMemcpyDeviceToHost, s));
  DI_CHECK(hipGetLastError());
  DI_CHECK(hipStreamSynchronize(s));  // nnzb; the temporaries go out of scope
  out.nnzb = in.pin[40];
  out.nent = (int)ne;
  out.ngrad = (int)ng;
  return 0;
}

}  // namespace yasps
