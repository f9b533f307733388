// Plan of the chunked symmetric SpMV over one part (static or dynamic) of the
// upper-triangular 3x3 BSR Hessian, built on the GPU from the part's row
// pointers and columns.
//
// The SpMV (pcg.hip) reads every stored upper block once.  The stored blocks
// are cut into chunks of CH consecutive blocks (row-major storage order); a
// workgroup takes a chunk, and each of its threads takes blocks of it in
// turn: for block (i, j) it forms B x_j for row i and, off the diagonal,
// B^T x_i for row j, and writes each product to its own LDS entry.  The
// entries of one target row are contiguous and in a fixed order (by block,
// the row product before the transposed one), so after a barrier each
// (chunk, target row) is summed by one thread and written to one slot of W;
// the slots of a row are contiguous, in chunk order, and the next kernel adds
// them.  No atomics: the result is bitwise reproducible.  This replaces the
// paper's atomic adds of the transposed products (appendix "SpMV", Algorithm
// "CUDA Block Level SpMV").
//
// Plan arrays (one part; m = compressed row: rows holding at least one block):
//   rl[m]          row id of compressed row m (null when every row holds blocks)
//   m0[c]          compressed row holding block c * CH
//   meta[k]        block k: its compressed row minus m0 of its chunk (bits 0-9),
//                  the LDS entry of its row product (bits 10-20) and of its
//                  transposed product (bits 21-31; unused on the diagonal)
//   tb[c]          first target of chunk c (tb[nchunk] = ntarget)
//   tend[t]        end of target t's LDS entries within its chunk
//   wslot[t]       W slot of target t
//   hptr[j]        W slots of row j: [hptr[j], hptr[j + 1])
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "devsort.h"
#include "kernels.h"

namespace yasps {

using namespace devsort;

namespace {

// per row r: 1 if it holds blocks
__global__ void plan_rows_kernel(int n, const int32_t* __restrict__ rp, int32_t* __restrict__ has) {
  const int r = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (r >= n) return;
  has[r] = rp[r + 1] > rp[r] ? 1 : 0;
}

// compressed rows, chunk heads, and the products to sort: block k's row
// product at 2k (key chunk of k << rbits | row), its transposed product at
// 2k + 1 (key chunk of k << rbits | column off the diagonal, the pad on it)
__global__ void plan_fill_kernel(int n, int ch, int rbits, uint64_t pad, const int32_t* __restrict__ rp,
                                 const int32_t* __restrict__ col, const int32_t* __restrict__ mpos,
                                 int32_t* __restrict__ rl, int32_t* __restrict__ m0, uint64_t* __restrict__ key,
                                 int32_t* __restrict__ val) {
  const int r = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (r >= n) return;
  const int a = rp[r], b = rp[r + 1];
  if (b <= a) return;
  const int m = mpos[r];
  rl[m] = r;
  for (int c = (a + ch - 1) / ch; c * ch < b; ++c) m0[c] = m;  // chunks whose first block lies in row r
  for (int k = a; k < b; ++k) {
    const uint64_t c = (uint64_t)(k / ch);
    const int j = col[k];
    key[2 * (size_t)k] = (c << rbits) | (uint64_t)r;
    val[2 * (size_t)k] = 2 * k;
    key[2 * (size_t)k + 1] = j != r ? ((c << rbits) | (uint64_t)j) : pad;
    val[2 * (size_t)k + 1] = 2 * k + 1;
  }
}

// first sorted entry of every chunk; 1 where a new (chunk, target) starts
__global__ void plan_starts_kernel(long long m, int rbits, const uint64_t* __restrict__ key, uint64_t pad,
                                   int32_t* __restrict__ cstart, int32_t* __restrict__ first) {
  const long long s = (long long)blockIdx.x * DI_BLOCK + threadIdx.x;
  if (s >= m) return;
  const uint64_t k = key[s];
  const bool real = k != pad;
  const bool head = real && (s == 0 || key[s - 1] != k);
  first[s] = head ? 1 : 0;
  if (real && (s == 0 || (key[s - 1] >> rbits) != (k >> rbits))) cstart[(int)(k >> rbits)] = (int)s;
}

// LDS entries of every product (into the packed block words), target ends,
// chunk target starts, target rows
__global__ void plan_place_kernel(long long m, int rbits, const uint64_t* __restrict__ key,
                                  const int32_t* __restrict__ val,
                                  uint64_t pad, const int32_t* __restrict__ cstart, const int32_t* __restrict__ tq,
                                  uint32_t* __restrict__ ypos, uint32_t* __restrict__ tpos,
                                  uint16_t* __restrict__ tend, int32_t* __restrict__ tb, int32_t* __restrict__ trow,
                                  int* max_entries) {
  const long long s = (long long)blockIdx.x * DI_BLOCK + threadIdx.x;
  if (s >= m) return;
  const uint64_t k = key[s];
  if (k == pad) return;
  const int c = (int)(k >> rbits);
  const int pos = (int)(s - cstart[c]);
  const int v = val[s];
  (v & 1 ? tpos : ypos)[v >> 1] = (uint32_t)pos;
  const int t = tq[s] - 1;
  if (s + 1 == m || key[s + 1] != k) {
    tend[t] = (uint16_t)(pos + 1);
    atomicMax(max_entries, pos + 1);
  }
  if (s == 0 || key[s - 1] != k) trow[t] = (int)(k & ((1ull << rbits) - 1));
  if (s == cstart[c]) tb[c] = t;
}

// meta[k] = local compressed row | row-product entry << 10 | transposed entry << 21
__global__ void plan_meta_kernel(int n, int ch, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                 const int32_t* __restrict__ mpos, const int32_t* __restrict__ m0,
                                 const uint32_t* __restrict__ ypos, const uint32_t* __restrict__ tpos,
                                 uint32_t* __restrict__ meta) {
  const int r = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (r >= n) return;
  const int a = rp[r], b = rp[r + 1];
  if (b <= a) return;
  const int m = mpos[r];
  for (int k = a; k < b; ++k) {
    const uint32_t lrow = (uint32_t)(m - m0[k / ch]);
    const uint32_t tp = col[k] != r ? tpos[k] : 0u;
    meta[k] = lrow | (ypos[k] << 10) | (tp << 21);
  }
}

__global__ void plan_iota_kernel(int m, int32_t* __restrict__ p) {
  const int i = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i < m) p[i] = i;
}

// W slots in (row, chunk) order: wslot[target] = its position in that order
__global__ void plan_wslot_kernel(int nt, const int32_t* __restrict__ tsorted, int32_t* __restrict__ wslot) {
  const int i = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (i < nt) wslot[tsorted[i]] = i;
}

// hptr[j] = first slot whose row is >= j (j = 0 .. n)
__global__ void plan_hptr_kernel(int n, int nt, const int32_t* __restrict__ rows, int32_t* __restrict__ hptr) {
  const int j = blockIdx.x * DI_BLOCK + threadIdx.x;
  if (j > n) return;
  int lo = 0, hi = nt;
  while (lo < hi) {
    const int mid = (lo + hi) / 2;
    if (rows[mid] < j)
      lo = mid + 1;
    else
      hi = mid;
  }
  hptr[j] = lo;
}

}  // namespace

int spmv_chunk_for(long long nblk) {
  if (const char* e = std::getenv("YASPS_SPMV_CHUNK")) {  // tuning override (a power of two, 64 .. SPMV_MAX_CHUNK)
    const int v = std::atoi(e);
    if (v >= 64 && v <= SPMV_MAX_CHUNK && (v & (v - 1)) == 0) return v;
  }
  long long c = 256;  // about 1024 chunks or more, up to SPMV_MAX_CHUNK blocks each
  while (c < SPMV_MAX_CHUNK && c * 2 * 1024 <= nblk) c *= 2;
  return (int)c;
}

#define PL_CHECK(expr)               \
  do {                               \
    const hipError_t e_ = (expr);    \
    if (e_ != hipSuccess) return -1; \
  } while (0)

int build_spmv_plan(int n, const int32_t* rp, const int32_t* col, int nblk, const void* vals, SpmvPart& out,
                    const std::function<void*(int, size_t)>& alloc, void* arena, size_t arena_bytes,
                    size_t* arena_needed, int* pin, hipStream_t s) {
  out = SpmvPart{};
  out.vals = vals;
  out.col = col;
  if (arena_needed) *arena_needed = 0;
  if (nblk == 0 || n == 0) return 0;
  const int ch = spmv_chunk_for(nblk);
  const int nchunk = (nblk + ch - 1) / ch;
  const long long m = 2ll * nblk;  // a row product and a transposed product (or the pad) per block
  const int rbits = bits_for(n);
  const uint64_t pad = (uint64_t)nchunk << rbits;
  const int kbits = rbits + bits_for(nchunk);
  Temp tmp;
  tmp.arena = static_cast<char*>(arena);
  tmp.cap = arena_bytes;
  struct Need {
    Temp& t;
    size_t* o;
    ~Need() {
      if (o) *o = t.used;
    }
  } need{tmp, arena_needed};
  int32_t* has = tmp.get<int32_t>(n);
  int32_t* mpos = tmp.get<int32_t>((size_t)n + 1);
  uint64_t* key = tmp.get<uint64_t>(m);
  uint64_t* key_s = tmp.get<uint64_t>(m);
  int32_t* val = tmp.get<int32_t>(m);
  int32_t* val_s = tmp.get<int32_t>(m);
  int32_t* cstart = tmp.get<int32_t>(nchunk);
  int32_t* first = tmp.get<int32_t>(m);
  int32_t* tq = tmp.get<int32_t>(m);
  uint32_t* ypos = tmp.get<uint32_t>(nblk);
  uint32_t* tpos = tmp.get<uint32_t>(nblk);
  int* scal = tmp.get<int>(4);
  PL_CHECK(tmp.err);
  auto ia = [&](int which, long long cnt) {
    return static_cast<int32_t*>(alloc(which, sizeof(int32_t) * (size_t)std::max<long long>(cnt, 1)));
  };
  int32_t* rl = ia(PL_RL, n);
  int32_t* m0 = ia(PL_M0, nchunk);
  int32_t* tb = ia(PL_TB, (long long)nchunk + 1);
  uint32_t* meta = static_cast<uint32_t*>(alloc(PL_META, sizeof(uint32_t) * (size_t)nblk));
  if (!rl || !m0 || !tb || !meta) return -1;

  hipLaunchKernelGGL(plan_rows_kernel, dim3(grid_of(n)), dim3(DI_BLOCK), 0, s, n, rp, has);
  PL_CHECK(prefix(tmp, has, mpos, n, s));
  hipLaunchKernelGGL(plan_fill_kernel, dim3(grid_of(n)), dim3(DI_BLOCK), 0, s, n, ch, rbits, pad, rp, col, mpos, rl,
                     m0, key, val);
  PL_CHECK(sort_pairs(tmp, key, key_s, val, val_s, m, kbits, s));
  PL_CHECK(hipMemsetAsync(scal, 0, 4 * sizeof(int), s));
  hipLaunchKernelGGL(plan_starts_kernel, dim3(grid_of(m)), dim3(DI_BLOCK), 0, s, m, rbits, key_s, pad, cstart,
                     first);
  PL_CHECK(inclusive(tmp, first, tq, m, s));
  int* head = pin;  // compressed rows, targets
  PL_CHECK(hipMemcpyAsync(&head[0], mpos + n, sizeof(int), hipMemcpyDeviceToHost, s));
  PL_CHECK(hipMemcpyAsync(&head[1], tq + (m - 1), sizeof(int), hipMemcpyDeviceToHost, s));
  PL_CHECK(hipStreamSynchronize(s));
  const int nt = head[1];
  uint16_t* tend = static_cast<uint16_t*>(alloc(PL_TEND, sizeof(uint16_t) * (size_t)std::max(nt, 1)));
  int32_t* wslot = ia(PL_WSLOT, nt);
  int32_t* hptr = ia(PL_HPTR, (long long)n + 1);
  int32_t* trow = tmp.get<int32_t>(nt);
  int32_t* trow_s = tmp.get<int32_t>(nt);
  int32_t* tid = tmp.get<int32_t>(nt);
  int32_t* tid_s = tmp.get<int32_t>(nt);
  PL_CHECK(tmp.err);
  if (!tend || !wslot || !hptr) return -1;
  hipLaunchKernelGGL(plan_place_kernel, dim3(grid_of(m)), dim3(DI_BLOCK), 0, s, m, rbits, key_s, val_s, pad, cstart,
                     tq, ypos, tpos, tend, tb, trow, scal);
  hipLaunchKernelGGL(plan_meta_kernel, dim3(grid_of(n)), dim3(DI_BLOCK), 0, s, n, ch, rp, col, mpos, m0, ypos, tpos,
                     meta);
  PL_CHECK(hipMemcpyAsync(tb + nchunk, &head[1], sizeof(int), hipMemcpyHostToDevice, s));
  // W slots: targets sorted stably by row (chunk order within a row)
  hipLaunchKernelGGL(plan_iota_kernel, dim3(grid_of(nt)), dim3(DI_BLOCK), 0, s, nt, tid);
  PL_CHECK(sort_pairs(tmp, trow, trow_s, tid, tid_s, nt, bits_for(n), s));
  hipLaunchKernelGGL(plan_wslot_kernel, dim3(grid_of(nt)), dim3(DI_BLOCK), 0, s, nt, tid_s, wslot);
  hipLaunchKernelGGL(plan_hptr_kernel, dim3(grid_of((long long)n + 1)), dim3(DI_BLOCK), 0, s, n, nt, trow_s, hptr);
  PL_CHECK(hipGetLastError());
  PL_CHECK(hipMemcpyAsync(pin + 2, scal, sizeof(int), hipMemcpyDeviceToHost, s));
  PL_CHECK(hipStreamSynchronize(s));  // the temporaries go out of scope
  const int max_entries = pin[2];
  out.nblk = nblk;
  out.nrows = head[0];
  out.nchunk = nchunk;
  out.ntarget = nt;
  out.chunk = ch;
  out.max_entries = max_entries;
  out.rl = head[0] == n ? nullptr : rl;  // every row holds blocks: the compressed rows are the rows
  out.m0 = m0;
  out.tb = tb;
  out.meta = meta;
  out.tend = tend;
  out.wslot = wslot;
  out.hptr = hptr;
  return 0;
}

}  // namespace yasps
