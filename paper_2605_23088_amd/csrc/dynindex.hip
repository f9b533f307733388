// Device build of the dynamic (contact) part's index structures: validation,
// storage order, block pattern and slot map, staging layout, and the SpMV's
// full row layout over the static and dynamic parts.
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

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace yasps {

namespace {

constexpr int DI_BLOCK = 256;

YDEV int verts_of(int t) { return t == 3 ? 2 : (t == 2 ? 3 : 4); }

int bits_for(long long v) {  // bits needed for values 0 .. v
  int b = 1;
  while ((1ll << b) <= v) ++b;
  return b;
}

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
                               int* counts) {
  const int j = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (j >= nc) return;
  const int s = order[j];
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

// Off-diagonal dynamic blocks keyed by (column, row) for the transposed
// entries of the full rows; the pad sorts last.
__global__ void transpose_keys_kernel(int nnzb, int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                      uint64_t pad, uint64_t* __restrict__ tkey, int32_t* __restrict__ tval) {
  const int r = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (r >= n) return;
  for (int k = rp[r]; k < rp[r + 1]; ++k) {
    const int c = col[k];
    tkey[k] = c != r ? (((uint64_t)c << 32) | (uint64_t)r) : pad;
    tval[k] = k;
  }
}

__global__ void transpose_count_kernel(int nt, const uint64_t* __restrict__ tkey, int32_t* __restrict__ tcnt) {
  const int i = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i >= nt) return;
  atomicAdd(&tcnt[(int)(tkey[i] >> 32)], 1);
}

// full row r: static share, dynamic upper blocks, dynamic transposed blocks
__global__ void full_count_kernel(int n, const int32_t* __restrict__ sf_ptr, const int32_t* __restrict__ rp,
                                  const int32_t* __restrict__ tptr, int32_t* __restrict__ fcnt) {
  const int r = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (r >= n) return;
  fcnt[r] = (sf_ptr[r + 1] - sf_ptr[r]) + (rp[r + 1] - rp[r]) + (tptr[r + 1] - tptr[r]);
}

__global__ void full_fill_kernel(int n, int nnzb_s, const int32_t* __restrict__ sf_ptr,
                                 const int32_t* __restrict__ sf_col, const int32_t* __restrict__ sf_src,
                                 const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                 const int32_t* __restrict__ tptr, const uint64_t* __restrict__ tkey,
                                 const int32_t* __restrict__ tval, const int32_t* __restrict__ f_rp,
                                 int32_t* __restrict__ f_col, int32_t* __restrict__ f_src) {
  const int r = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (r >= n) return;
  int p = f_rp[r];
  for (int k = sf_ptr[r]; k < sf_ptr[r + 1]; ++k, ++p) {
    f_col[p] = sf_col[k];
    f_src[p] = sf_src[k];
  }
  for (int k = rp[r]; k < rp[r + 1]; ++k, ++p) {
    f_col[p] = col[k];
    f_src[p] = nnzb_s + k;
  }
  for (int t = tptr[r]; t < tptr[r + 1]; ++t, ++p) {
    f_col[p] = (int)(tkey[t] & 0xffffffffu);
    f_src[p] = -(nnzb_s + tval[t]) - 1;
  }
}

// first row of each XCD range: work(r) = f_rp[r] + row_cost r reaches x / PCG_XCDS of the total
__global__ void xsplit_kernel(int n, const int32_t* __restrict__ f_rp, int row_cost, int* xsplit) {
  const int x = threadIdx.x;
  if (x > PCG_XCDS) return;
  const long long work = (long long)f_rp[n] + (long long)row_cost * n;
  const long long target = work * x / PCG_XCDS;
  int lo = 0, hi = n;  // smallest r with f_rp[r] + row_cost r >= target
  while (lo < hi) {
    const int mid = (lo + hi) / 2;
    if ((long long)f_rp[mid] + (long long)row_cost * mid < target)
      lo = mid + 1;
    else
      hi = mid;
  }
  xsplit[x] = x == PCG_XCDS ? n : lo;
}

__global__ void fill_i32_kernel(long long m, int32_t v, int32_t* __restrict__ p) {
  const long long i = (long long)blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i < m) p[i] = v;
}

__global__ void iota_kernel(int m, int32_t* __restrict__ p) {
  const int i = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i < m) p[i] = i;
}

int grid_of(long long m) { return (int)std::max<long long>(1, (m + DI_BLOCK - 1) / DI_BLOCK); }

// Temporaries of one build, carved from the caller's arena while it lasts
// (256-byte aligned), else allocated and freed when done; `used` is the arena
// size the whole build needs.
struct Temp {
  char* arena = nullptr;
  size_t cap = 0, used = 0;
  std::vector<void*> ptrs;
  hipError_t err = hipSuccess;
  template <class T>
  T* get(size_t count) {
    const size_t bytes = (std::max<size_t>(count, 1) * sizeof(T) + 255) / 256 * 256;
    void* p = nullptr;
    if (used + bytes <= cap) {
      p = arena + used;
    } else if (err == hipSuccess) {
      err = hipMalloc(&p, bytes);
      if (p) ptrs.push_back(p);
    }
    used += bytes;
    return static_cast<T*>(p);
  }
  ~Temp() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

template <class K, class V>
hipError_t sort_pairs(Temp& tmp, const K* ki, K* ko, const V* vi, V* vo, long long m, int end_bit, hipStream_t s) {
  if (m == 0) return hipSuccess;
  size_t bytes = 0;
  hipError_t e = rocprim::radix_sort_pairs(nullptr, bytes, ki, ko, vi, vo, (size_t)m, 0u, (unsigned)end_bit, s);
  if (e != hipSuccess) return e;
  void* store = tmp.get<char>(bytes);
  if (tmp.err != hipSuccess) return tmp.err;
  return rocprim::radix_sort_pairs(store, bytes, ki, ko, vi, vo, (size_t)m, 0u, (unsigned)end_bit, s);
}

// out[0] = 0, out[k + 1] = in[0] + ... + in[k]  (k < m)
hipError_t prefix(Temp& tmp, const int32_t* in, int32_t* out, long long m, hipStream_t s) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(int32_t), s);
  if (e != hipSuccess || m == 0) return e;
  size_t bytes = 0;
  e = rocprim::inclusive_scan(nullptr, bytes, in, out + 1, (size_t)m, rocprim::plus<int32_t>(), s);
  if (e != hipSuccess) return e;
  void* store = tmp.get<char>(bytes);
  if (tmp.err != hipSuccess) return tmp.err;
  return rocprim::inclusive_scan(store, bytes, in, out + 1, (size_t)m, rocprim::plus<int32_t>(), s);
}

hipError_t inclusive(Temp& tmp, const int32_t* in, int32_t* out, long long m, hipStream_t s) {
  if (m == 0) return hipSuccess;
  size_t bytes = 0;
  hipError_t e = rocprim::inclusive_scan(nullptr, bytes, in, out, (size_t)m, rocprim::plus<int32_t>(), s);
  if (e != hipSuccess) return e;
  void* store = tmp.get<char>(bytes);
  if (tmp.err != hipSuccess) return tmp.err;
  return rocprim::inclusive_scan(store, bytes, in, out, (size_t)m, rocprim::plus<int32_t>(), s);
}

// Far entries: per row, the entries below the diagonal whose stored block is
// a contact block (at or above nnzb_s) more than far_rows rows back.
YDEV bool far_entry(int32_t sk, int r, int c, int nnzb_s, int far_rows) {
  return sk < 0 && -sk - 1 >= nnzb_s && r - c > far_rows;
}

__global__ __launch_bounds__(DI_BLOCK) void far_count_kernel(int n, int nnzb_s, int far_rows,
                                                             const int32_t* __restrict__ f_rp,
                                                             const int32_t* __restrict__ f_col,
                                                             const int32_t* __restrict__ f_src,
                                                             int32_t* __restrict__ cnt) {
  const int r = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (r >= n) return;
  int c = 0;
  for (int k = f_rp[r]; k < f_rp[r + 1]; ++k) c += far_entry(f_src[k], r, f_col[k], nnzb_s, far_rows);
  cnt[r] = c;
}

// Row by row, in entry order: far copy j gets the stored block, the entry
// the code nnzb_total + j.
__global__ __launch_bounds__(DI_BLOCK) void far_fill_kernel(int n, int nnzb_s, int far_rows, int nnzb_total,
                                                            const int32_t* __restrict__ f_rp,
                                                            const int32_t* __restrict__ f_col,
                                                            int32_t* __restrict__ f_src,
                                                            const int32_t* __restrict__ ptr,
                                                            int32_t* __restrict__ far_src) {
  const int r = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (r >= n) return;
  int j = ptr[r];
  for (int k = f_rp[r]; k < f_rp[r + 1]; ++k) {
    const int32_t sk = f_src[k];
    if (far_entry(sk, r, f_col[k], nnzb_s, far_rows)) {
      far_src[j] = -sk - 1;
      f_src[k] = nnzb_total + j;
      ++j;
    }
  }
}

}  // namespace

#define DI_CHECK(expr)                       \
  do {                                       \
    const hipError_t e_ = (expr);            \
    if (e_ != hipSuccess) return -1;         \
  } while (0)

int split_far_entries(int n, const int32_t* f_rp, const int32_t* f_col, int32_t* f_src, int nnzb_s, int nnzb_total,
                      int far_rows, int32_t** far_src, int* nfar, const std::function<void*(size_t)>& alloc,
                      hipStream_t s) {
  *far_src = nullptr;
  *nfar = 0;
  if (n == 0) return 0;
  Temp tmp;
  int32_t* cnt = tmp.get<int32_t>(n);
  int32_t* ptr = tmp.get<int32_t>((size_t)n + 1);
  if (tmp.err != hipSuccess) return -1;
  hipLaunchKernelGGL(far_count_kernel, dim3(grid_of(n)), dim3(DI_BLOCK), 0, s, n, nnzb_s, far_rows, f_rp, f_col,
                     f_src, cnt);
  DI_CHECK(prefix(tmp, cnt, ptr, n, s));
  int total = 0;
  DI_CHECK(hipMemcpyAsync(&total, ptr + n, sizeof(int), hipMemcpyDeviceToHost, s));
  DI_CHECK(hipStreamSynchronize(s));
  if (total == 0) return 0;
  *far_src = static_cast<int32_t*>(alloc((size_t)total * sizeof(int32_t)));
  if (!*far_src) return -1;
  hipLaunchKernelGGL(far_fill_kernel, dim3(grid_of(n)), dim3(DI_BLOCK), 0, s, n, nnzb_s, far_rows, nnzb_total, f_rp,
                     f_col, f_src, ptr, *far_src);
  DI_CHECK(hipGetLastError());
  DI_CHECK(hipStreamSynchronize(s));  // the temporaries are freed on return
  *nfar = total;
  return 0;
}

int build_dynamic_index(const DynIndexIn& in, DynIndexOut& out, const std::function<void*(size_t)>& alloc,
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
  // small device scalars: err, counts[2] (block / gradient entries), offdiag, gcount[32], xsplit[9]
  int* scal = tmp.get<int>(48);
  DI_CHECK(tmp.err);
  int* err = scal;
  int* counts = scal + 1;
  int* offdiag = scal + 3;
  int* gcount = scal + 4;
  int* xsplit = scal + 36;
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
  int32_t* sidx = static_cast<int32_t*>(alloc(sizeof(int32_t) * std::max<long long>(nge, 1)));
  DI_CHECK(tmp.err);
  if (!sidx) return -1;
  if (nc) {
    hipLaunchKernelGGL(entries_kernel, dim3(grid_of(nc)), dim3(DI_BLOCK), 0, s, nc, n, in.idx, order, bpad, sidx,
                       bkey, bval, gkey, gval, counts);
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
  auto ialloc = [&](long long m) { return static_cast<int32_t*>(alloc(sizeof(int32_t) * std::max<long long>(m, 1))); };
  out.rp = ialloc(n + 1);
  out.col = ialloc(nnzb);
  out.cptr = ialloc(nnzb + 1);
  out.slot = ialloc(10ll * nc);
  out.spos = ialloc(10ll * nc);
  out.gpos = ialloc(4ll * nc);
  out.gptr = ialloc(n + 1);
  out.ddiag = ialloc(n);
  out.sidx = sidx;
  if (!out.rp || !out.col || !out.cptr || !out.slot || !out.spos || !out.gpos || !out.gptr || !out.ddiag) return -1;
  int32_t* rowcnt = tmp.get<int32_t>(n);
  DI_CHECK(tmp.err);
  DI_CHECK(hipMemsetAsync(rowcnt, 0, sizeof(int32_t) * std::max(n, 1), s));
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_of(10ll * nc)), dim3(DI_BLOCK), 0, s, 10ll * nc, -1, out.slot);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_of(10ll * nc)), dim3(DI_BLOCK), 0, s, 10ll * nc, -1, out.spos);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_of(4ll * nc)), dim3(DI_BLOCK), 0, s, 4ll * nc, -1, out.gpos);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_of(n)), dim3(DI_BLOCK), 0, s, (long long)n, -1, out.ddiag);
  if (ne)
    hipLaunchKernelGGL(blocks_kernel, dim3(grid_of(ne)), dim3(DI_BLOCK), 0, s, ne, nc, bkey_s, bval_s, blk, first,
                       order, out.spos, out.col, out.cptr, out.slot, rowcnt, out.ddiag, offdiag);
  DI_CHECK(hipMemcpyAsync(out.cptr + nnzb, &ne, sizeof(int), hipMemcpyHostToDevice, s));
  DI_CHECK(prefix(tmp, rowcnt, out.rp, n, s));
  if (ng) hipLaunchKernelGGL(grads_kernel, dim3(grid_of(ng)), dim3(DI_BLOCK), 0, s, ng, nc, gval_s, out.gpos);
  hipLaunchKernelGGL(gptr_kernel, dim3(grid_of(n + 1)), dim3(DI_BLOCK), 0, s, n, ng, gkey_s, out.gptr);

  // 4. transposed dynamic blocks (sorted by column, then row) and the full rows
  uint64_t* tkey = tmp.get<uint64_t>(nnzb);
  uint64_t* tkey_s = tmp.get<uint64_t>(nnzb);
  int32_t* tval = tmp.get<int32_t>(nnzb);
  int32_t* tval_s = tmp.get<int32_t>(nnzb);
  int32_t* tcnt = tmp.get<int32_t>(n);
  int32_t* tptr = tmp.get<int32_t>(n + 1);
  int32_t* fcnt = tmp.get<int32_t>(n);
  DI_CHECK(tmp.err);
  DI_CHECK(hipMemsetAsync(tcnt, 0, sizeof(int32_t) * std::max(n, 1), s));
  int noff = 0;
  DI_CHECK(hipMemcpyAsync(&noff, offdiag, sizeof(int), hipMemcpyDeviceToHost, s));
  DI_CHECK(hipStreamSynchronize(s));
  if (nnzb) {
    hipLaunchKernelGGL(transpose_keys_kernel, dim3(grid_of(n)), dim3(DI_BLOCK), 0, s, nnzb, n, out.rp, out.col, bpad,
                       tkey, tval);
    DI_CHECK(sort_pairs(tmp, tkey, tkey_s, tval, tval_s, nnzb, 32 + nbits, s));
    if (noff) hipLaunchKernelGGL(transpose_count_kernel, dim3(grid_of(noff)), dim3(DI_BLOCK), 0, s, noff, tkey_s, tcnt);
  }
  DI_CHECK(prefix(tmp, tcnt, tptr, n, s));
  if (n) hipLaunchKernelGGL(full_count_kernel, dim3(grid_of(n)), dim3(DI_BLOCK), 0, s, n, in.sf_ptr, out.rp, tptr, fcnt);
  out.f_rp = ialloc(n + 1);
  if (!out.f_rp) return -1;
  DI_CHECK(prefix(tmp, fcnt, out.f_rp, n, s));
  const long long f_nnz = (long long)in.sf_nnz + nnzb + noff;
  out.f_col = ialloc(f_nnz);
  out.f_src = ialloc(f_nnz);
  if (!out.f_col || !out.f_src) return -1;
  if (n)
    hipLaunchKernelGGL(full_fill_kernel, dim3(grid_of(n)), dim3(DI_BLOCK), 0, s, n, in.nnzb_s, in.sf_ptr, in.sf_col,
                       in.sf_src, out.rp, out.col, tptr, tkey_s, tval_s, out.f_rp, out.f_col, out.f_src);
  hipLaunchKernelGGL(xsplit_kernel, dim3(1), dim3(64), 0, s, n, out.f_rp, in.row_cost, xsplit);
  DI_CHECK(hipGetLastError());
  DI_CHECK(hipMemcpyAsync(out.xsplit, xsplit, sizeof(out.xsplit), hipMemcpyDeviceToHost, s));
  DI_CHECK(hipStreamSynchronize(s));
  out.nnzb = nnzb;
  out.nent = ne;
  out.ngrad = ng;
  out.f_nnz = f_nnz;
  return 0;
}

}  // namespace yasps
