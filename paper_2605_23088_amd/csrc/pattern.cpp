// Host-side pattern, slot map and staging layout (see pattern.h).
#include "pattern.h"

#include <algorithm>
#include <numeric>

namespace yasps {

int used_vertices(const int32_t* idx, int ns, int s, int width) {
  int k = 0;
  for (int a = 0; a < width; ++a)
    if (idx[a * (size_t)ns + s] >= 0) ++k;
  return k;
}

void build_pattern(int n, const int32_t* idx, int ns, bool diag, PartPattern& out, int width) {
  const int np = width * (width + 1) / 2;
  std::vector<uint64_t> keys;
  keys.reserve((size_t)ns * np + (diag ? n : 0));
  for (int s = 0; s < ns; ++s) {
    const int k = used_vertices(idx, ns, s, width);
    for (int a = 0; a < k; ++a)
      for (int b = a; b < k; ++b) {
        const int va = idx[a * (size_t)ns + s], vb = idx[b * (size_t)ns + s];
        if (va < n && vb < n) {
          const uint64_t r = (uint64_t)std::min(va, vb), c = (uint64_t)std::max(va, vb);
          keys.push_back((r << 32) | c);
        }
      }
  }
  if (diag)
    for (int v = 0; v < n; ++v) keys.push_back(((uint64_t)v << 32) | (uint64_t)v);
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  out.nnzb = (int)keys.size();
  out.row_ptr.assign(n + 1, 0);
  out.col_idx.resize(keys.size());
  for (size_t i = 0; i < keys.size(); ++i) {
    out.row_ptr[(keys[i] >> 32) + 1]++;
    out.col_idx[i] = (int32_t)(keys[i] & 0xffffffffu);
  }
  for (int v = 0; v < n; ++v) out.row_ptr[v + 1] += out.row_ptr[v];
  out.slot.assign((size_t)ns * np, -1);
  for (int s = 0; s < ns; ++s) {
    const int k = used_vertices(idx, ns, s, width);
    int q = 0;
    for (int a = 0; a < k; ++a)
      for (int b = a; b < k; ++b, ++q) {
        const int va = idx[a * (size_t)ns + s], vb = idx[b * (size_t)ns + s];
        if (va < n && vb < n) {
          const int r = std::min(va, vb), c = std::max(va, vb);
          const int32_t* lo = out.col_idx.data() + out.row_ptr[r];
          const int32_t* hi = out.col_idx.data() + out.row_ptr[r + 1];
          out.slot[(size_t)s * np + q] = (int32_t)(std::lower_bound(lo, hi, c) - out.col_idx.data());
        }
      }
  }
}

void build_staging(int n, const int32_t* idx, int ns, const PartPattern& pat, const std::vector<int32_t>& order,
                   bool lead_block, bool lead_grad, Staging& st, int width, int nlead) {
  const int np = width * (width + 1) / 2;
  if (nlead < 0) nlead = n;
  const int nnzb = pat.nnzb;
  std::vector<int32_t> cnt(nnzb, 0), gcnt(n, 0);
  if (lead_block)
    for (int v = 0; v < nlead; ++v) cnt[pat.row_ptr[v]]++;  // diagonal block is first in its row
  if (lead_grad)
    for (int v = 0; v < nlead; ++v) gcnt[v]++;
  for (int s = 0; s < ns; ++s) {
    for (int q = 0; q < np; ++q) {
      const int32_t sl = pat.slot[(size_t)s * np + q];
      if (sl >= 0) cnt[sl]++;
    }
    for (int a = 0; a < width; ++a) {
      const int v = idx[a * (size_t)ns + s];
      if (v >= 0 && v < n) gcnt[v]++;
    }
  }
  st.cptr.assign(nnzb + 1, 0);
  for (int k = 0; k < nnzb; ++k) st.cptr[k + 1] = st.cptr[k] + cnt[k];
  st.gptr.assign(n + 1, 0);
  for (int v = 0; v < n; ++v) st.gptr[v + 1] = st.gptr[v] + gcnt[v];
  st.nblocks = st.cptr[nnzb];
  st.ngrads = st.gptr[n];
  std::vector<int32_t> fill(st.cptr.begin(), st.cptr.end() - 1), gfill(st.gptr.begin(), st.gptr.end() - 1);
  st.lead_spos.assign(nlead, -1);
  st.lead_gpos.assign(nlead, -1);
  if (lead_block)
    for (int v = 0; v < nlead; ++v) st.lead_spos[v] = fill[pat.row_ptr[v]]++;
  if (lead_grad)
    for (int v = 0; v < nlead; ++v) st.lead_gpos[v] = gfill[v]++;
  // positions are stored in storage order: spos[q][j], j = position of the stencil in `order`
  st.spos.assign((size_t)np * ns, -1);
  st.gpos.assign((size_t)width * ns, -1);
  for (int j = 0; j < ns; ++j) {
    const int s = order[j];
    for (int q = 0; q < np; ++q) {
      const int32_t sl = pat.slot[(size_t)s * np + q];
      if (sl >= 0) st.spos[(size_t)q * ns + j] = fill[sl]++;
    }
    for (int a = 0; a < width; ++a) {
      const int v = idx[a * (size_t)ns + s];
      if (v >= 0 && v < n) st.gpos[(size_t)a * ns + j] = gfill[v]++;
    }
  }
}

}  // namespace yasps
