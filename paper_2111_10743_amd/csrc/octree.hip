// Device build of the uniform-depth octree (Octree::build_device): the same
// tree as the host build (octree.cpp) -- frame, depth, stable orders of the
// targets and sources by leaf key, boxes per level, parent/child links,
// U-lists and V-lists -- computed by HIP kernels:
//   Morton keys (21 bits per axis) -> stable LSD radix sorts (8-bit digits,
//   per-block histograms, one exclusive scan, rank-preserving scatter) ->
//   unique prefixes per level (flag + scan + compact) -> binary-search links
//   and lists (count + scan + fill).
// Only the few scalars that choose the frame and the depth pass through the
// host; the results are copied into the host-side Octree at the end.
#include "octree.hpp"
#include "common.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace lb {

#define OCHK(x)                                                                              \
  do {                                                                                       \
    hipError_t e_ = (x);                                                                     \
    if (e_ != hipSuccess) fail(LB_EHIP, "octree: %s: %s", #x, hipGetErrorString(e_));       \
  } while (0)
#define OKCHK() OCHK(hipGetLastError())

namespace {

template <typename T>
struct DVec {
  T* p = nullptr;
  size_t n = 0;
  DVec() = default;
  explicit DVec(size_t m) { alloc(m); }
  DVec(const DVec&) = delete;
  DVec& operator=(const DVec&) = delete;
  ~DVec() {
    if (p) (void)hipFree(p);
  }
  void alloc(size_t m) {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = m;
    if (m) OCHK(hipMalloc(&p, sizeof(T) * m));
  }
  std::vector<T> host(size_t m) const {
    std::vector<T> h(m);
    if (m) OCHK(hipMemcpy(h.data(), p, sizeof(T) * m, hipMemcpyDeviceToHost));
    return h;
  }
};

__device__ inline uint64_t d_spread21(uint64_t x) {
  x &= 0x1fffff;
  x = (x | x << 32) & 0x1f00000000ffffULL;
  x = (x | x << 16) & 0x1f0000ff0000ffULL;
  x = (x | x << 8) & 0x100f00f00f00f00fULL;
  x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
  x = (x | x << 2) & 0x1249249249249249ULL;
  return x;
}
__device__ inline uint64_t d_morton(uint64_t ix, uint64_t iy, uint64_t iz) {
  return d_spread21(ix) | (d_spread21(iy) << 1) | (d_spread21(iz) << 2);
}
__device__ inline int d_compact21(uint64_t x) {
  x &= 0x1249249249249249ULL;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ULL;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00fULL;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffULL;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffULL;
  x = (x ^ (x >> 32)) & 0x1fffff;
  return (int)x;
}

// index of key k in the sorted unique array a[0..n), or -1
__device__ inline int d_find(const uint64_t* a, int n, uint64_t k) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < k) lo = mid + 1; else hi = mid;
  }
  return (lo < n && a[lo] == k) ? lo : -1;
}
// first index of a sorted array a[0..n) with a[i] >= k (upper: > k)
__device__ inline int64_t d_lower(const uint64_t* a, int64_t n, uint64_t k) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < k) lo = mid + 1; else hi = mid;
  }
  return lo;
}
__device__ inline int64_t d_upper(const uint64_t* a, int64_t n, uint64_t k) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] <= k) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// ---- bounding box: per-block min/max of x, y, z over both point sets ----
__global__ void k_minmax(const double* __restrict__ a, int64_t na, const double* __restrict__ b, int64_t nb,
                         double* __restrict__ part) {
  __shared__ double s[6][256];
  double v[6] = {1e300, 1e300, 1e300, -1e300, -1e300, -1e300};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < na + nb; i += (int64_t)gridDim.x * 256) {
    const double* p = i < na ? a + 3 * i : b + 3 * (i - na);
    for (int d = 0; d < 3; ++d) {
      v[d] = fmin(v[d], p[d]);
      v[3 + d] = fmax(v[3 + d], p[d]);
    }
  }
  for (int d = 0; d < 6; ++d) s[d][threadIdx.x] = v[d];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int d = 0; d < 6; ++d)
        s[d][threadIdx.x] = d < 3 ? fmin(s[d][threadIdx.x], s[d][threadIdx.x + o])
                                  : fmax(s[d][threadIdx.x], s[d][threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

// ---- Morton keys with the host build's arithmetic ----
__global__ void k_keys(const double* __restrict__ p, int64_t n, double lo0, double lo1, double lo2, double scale,
                       uint64_t* __restrict__ key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lo[3] = {lo0, lo1, lo2};
  uint64_t c[3];
  for (int d = 0; d < 3; ++d) {
    const double t = floor((p[3 * i + d] - lo[d]) * scale);
    c[d] = (uint64_t)fmin(fmax(t, 0.0), (double)((1 << 21) - 1));
  }
  key[i] = d_morton(c[0], c[1], c[2]);
}

__global__ void k_iota(int* v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (int)i;
}

__global__ void k_shift(const uint64_t* __restrict__ a, int64_t n, int s, uint64_t* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i] >> s;
}

// ---- exclusive scan of int32 counts, one block of 1024 threads (setup
// sizes: a thread owns a contiguous segment); total -> *tot ----
__global__ __launch_bounds__(1024) void k_scan(const int* __restrict__ in, int* __restrict__ out, int64_t n,
                                               int* __restrict__ tot) {
  __shared__ long long s[1024];
  const int64_t seg = (n + 1023) / 1024;
  const int64_t b = threadIdx.x * seg, e = min(n, b + seg);
  long long a = 0;
  for (int64_t i = b; i < e; ++i) a += in[i];
  s[threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long r = 0;
    for (int t = 0; t < 1024; ++t) {
      const long long v = s[t];
      s[t] = r;
      r += v;
    }
    *tot = (int)r;
  }
  __syncthreads();
  long long r = s[threadIdx.x];
  for (int64_t i = b; i < e; ++i) {
    const int v = in[i];
    out[i] = (int)r;
    r += v;
  }
}

// ---- stable LSD radix sort by 8-bit digits ----
constexpr int RS_TILE = 4096;  // elements per block (16 chunks of 256)

__global__ __launch_bounds__(256) void k_rs_hist(const uint64_t* __restrict__ key, int64_t n, int shift,
                                                 int* __restrict__ hist, int nblk) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t b = (int64_t)blockIdx.x * RS_TILE;
  for (int c = 0; c < RS_TILE / 256; ++c) {
    const int64_t i = b + c * 256 + threadIdx.x;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// The tile is taken in order in chunks of 256; within a chunk the rank of an
// element among the equal digits before it comes from ballots (wave) and
// per-wave digit counts (block); `run` carries the block's next free slot
// per digit from chunk to chunk.  Hence equal digits keep their order.
__global__ __launch_bounds__(256) void k_rs_scatter(const uint64_t* __restrict__ kin, const int* __restrict__ vin,
                                                    uint64_t* __restrict__ kout, int* __restrict__ vout, int64_t n,
                                                    int shift, const int* __restrict__ offs, int nblk) {
  __shared__ int run[256];
  __shared__ int wc[4][257];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  run[threadIdx.x] = offs[(int64_t)threadIdx.x * nblk + blockIdx.x];
  const int64_t b = (int64_t)blockIdx.x * RS_TILE;
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (int c = 0; c < RS_TILE / 256; ++c) {
    const int64_t i = b + c * 256 + threadIdx.x;
    const bool valid = i < n;
    uint64_t k = 0;
    int v = 0;
    if (valid) { k = kin[i]; v = vin[i]; }
    const int dig = valid ? (int)((k >> shift) & 255) : 256;
    unsigned long long peers = __ballot(valid);
    if (!valid) peers = ~peers;
    for (int bit = 0; bit < 8; ++bit) {
      const unsigned long long bl = __ballot((dig >> bit) & 1);
      peers &= ((dig >> bit) & 1) ? bl : ~bl;
    }
    const int rk = __popcll(peers & lt);
    for (int q = threadIdx.x; q < 4 * 257; q += 256) (&wc[0][0])[q] = 0;
    __syncthreads();
    if (rk == 0) wc[w][dig] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = run[dig] + rk;
      for (int ww = 0; ww < w; ++ww) pos += wc[ww][dig];
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    run[threadIdx.x] += wc[0][threadIdx.x] + wc[1][threadIdx.x] + wc[2][threadIdx.x] + wc[3][threadIdx.x];
    __syncthreads();
  }
}

// sort (key, val) pairs by bits [0, bits) of key, stably; in/out buffers swap
void radix_sort(DVec<uint64_t>& key, DVec<int>& val, int64_t n, int bits) {
  if (n <= 1 || bits <= 0) return;
  const int nblk = (int)((n + RS_TILE - 1) / RS_TILE);
  DVec<uint64_t> k2(n);
  DVec<int> v2(n), hist((size_t)256 * nblk), offs((size_t)256 * nblk), tot(1);
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(256), 0, 0, key.p, n, shift, hist.p, nblk);
    OKCHK();
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, 0, hist.p, offs.p, (int64_t)256 * nblk, tot.p);
    OKCHK();
    hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(256), 0, 0, key.p, val.p, k2.p, v2.p, n, shift, offs.p, nblk);
    OKCHK();
    std::swap(key.p, k2.p);
    std::swap(val.p, v2.p);
  }
}

// ---- unique run heads of a sorted key array -> compacted keys ----
__global__ void k_heads(const uint64_t* __restrict__ a, int64_t n, int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = (i == 0 || a[i] != a[i - 1]) ? 1 : 0;
}
__global__ void k_compact(const uint64_t* __restrict__ a, int64_t n, const int* __restrict__ flag,
                          const int* __restrict__ pos, uint64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = a[i];
}

// counts of distinct prefixes (key >> 3 (21 - l)) of a sorted key array,
// l = 2..20: per-block partial counts part[blk][l]
__global__ void k_level_counts(const uint64_t* __restrict__ a, int64_t n, int* __restrict__ part) {
  __shared__ int c[21];
  if (threadIdx.x < 21) c[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n)
    for (int l = 2; l <= 20; ++l) {
      const int s = 3 * (21 - l);
      if (i == 0 || (a[i] >> s) != (a[i - 1] >> s)) atomicAdd(&c[l], 1);
    }
  __syncthreads();
  if (threadIdx.x < 21) part[(int64_t)blockIdx.x * 21 + threadIdx.x] = c[threadIdx.x];
}

// ---- boxes: coordinates, parent/child links (global ids) ----
__global__ void k_boxes(const uint64_t* __restrict__ keys, const int* __restrict__ lev_off, int depth, int nb,
                        int* __restrict__ bx, int* __restrict__ by, int* __restrict__ bz, int* __restrict__ parent,
                        int* __restrict__ child) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nb) return;
  int l = 0;
  while (g >= lev_off[l + 1]) ++l;
  const uint64_t k = keys[g];
  bx[g] = d_compact21(k);
  by[g] = d_compact21(k >> 1);
  bz[g] = d_compact21(k >> 2);
  if (l > 0) {
    const int pl = d_find(keys + lev_off[l - 1], lev_off[l] - lev_off[l - 1], k >> 3);
    const int pg = lev_off[l - 1] + pl;  // always present: levels are built from their children
    parent[g] = pg;
    child[(int64_t)pg * 8 + (k & 7)] = g;
  } else {
    parent[g] = -1;
  }
}

// leaf ranges in the sorted leaf-key arrays of targets and sources
__global__ void k_leaf_ranges(const uint64_t* __restrict__ lk, int nleaf, const uint64_t* __restrict__ tk,
                              int64_t nt, const uint64_t* __restrict__ sk, int64_t ns, int* __restrict__ tb,
                              int* __restrict__ te, int* __restrict__ sb, int* __restrict__ se,
                              unsigned char* __restrict__ hs, unsigned char* __restrict__ ht, int leaf_off) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  const uint64_t k = lk[b];
  tb[b] = (int)d_lower(tk, nt, k);
  te[b] = (int)d_upper(tk, nt, k);
  sb[b] = (int)d_lower(sk, ns, k);
  se[b] = (int)d_upper(sk, ns, k);
  ht[leaf_off + b] = te[b] > tb[b];
  hs[leaf_off + b] = se[b] > sb[b];
}

// has flags of level l from its children
__global__ void k_has_up(const int* __restrict__ child, int g0, int g1, unsigned char* __restrict__ hs,
                         unsigned char* __restrict__ ht) {
  const int g = g0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= g1) return;
  unsigned char a = 0, b = 0;
  for (int c = 0; c < 8; ++c) {
    const int ch = child[(int64_t)g * 8 + c];
    if (ch >= 0) { a |= hs[ch]; b |= ht[ch]; }
  }
  hs[g] = a;
  ht[g] = b;
}

__device__ inline int d_lookup(const uint64_t* keys, const int* lev_off, int l, int x, int y, int z) {
  const int n = 1 << l;
  if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) return -1;
  const int i = d_find(keys + lev_off[l], lev_off[l + 1] - lev_off[l], d_morton(x, y, z));
  return i < 0 ? -1 : lev_off[l] + i;
}

// U-lists of the leaves holding targets: adjacent leaves holding sources, in
// the (dx, dy, dz) loop order of the host build.  FILL = false counts.
template <bool FILL>
__global__ void k_ulist(const uint64_t* __restrict__ keys, const int* __restrict__ lev_off, int depth, int nleaf,
                        const int* __restrict__ bx, const int* __restrict__ by, const int* __restrict__ bz,
                        const unsigned char* __restrict__ hs, const unsigned char* __restrict__ ht,
                        int* __restrict__ cnt, const int* __restrict__ ptr, int* __restrict__ list) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nleaf) return;
  const int g = lev_off[depth] + b;
  int c = 0;
  if (ht[g])
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          const int nbx = d_lookup(keys, lev_off, depth, bx[g] + dx, by[g] + dy, bz[g] + dz);
          if (nbx >= 0 && hs[nbx]) {
            if (FILL) list[ptr[b] + c] = nbx - lev_off[depth];
            ++c;
          }
        }
  if (!FILL) cnt[b] = c;
}

// V-lists of the boxes holding targets on levels >= 2: children of the
// parent's neighbours that hold sources and are not adjacent; offset id
// ((ox+3)*7 + (oy+3))*7 + (oz+3) of (target - source) in box units.
template <bool FILL>
__global__ void k_vlist(const uint64_t* __restrict__ keys, const int* __restrict__ lev_off, int nb,
                        const int* __restrict__ bx, const int* __restrict__ by, const int* __restrict__ bz,
                        const int* __restrict__ parent, const int* __restrict__ child,
                        const unsigned char* __restrict__ hs, const unsigned char* __restrict__ ht,
                        int* __restrict__ cnt, const int* __restrict__ ptr, int* __restrict__ vsrc,
                        int* __restrict__ voff) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nb) return;
  int l = 0;
  while (g >= lev_off[l + 1]) ++l;
  int c = 0;
  if (l >= 2 && ht[g]) {
    const int pg = parent[g];
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          const int pn = d_lookup(keys, lev_off, l - 1, bx[pg] + dx, by[pg] + dy, bz[pg] + dz);
          if (pn < 0) continue;
          for (int q = 0; q < 8; ++q) {
            const int ch = child[(int64_t)pn * 8 + q];
            if (ch < 0 || !hs[ch]) continue;
            const int ox = bx[g] - bx[ch], oy = by[g] - by[ch], oz = bz[g] - bz[ch];
            if (abs(ox) <= 1 && abs(oy) <= 1 && abs(oz) <= 1) continue;
            if (FILL) {
              vsrc[ptr[g] + c] = ch;
              voff[ptr[g] + c] = ((ox + 3) * 7 + (oy + 3)) * 7 + (oz + 3);
            }
            ++c;
          }
        }
  }
  if (!FILL) cnt[g] = c;
}

inline dim3 grid_for(int64_t n, int bs = 256) { return dim3((unsigned)std::max<int64_t>(1, (n + bs - 1) / bs)); }

// exclusive scan of n counts into ptr[0..n], returns the total
int scan_counts(const DVec<int>& cnt, int64_t n, DVec<int>& ptr) {
  ptr.alloc(n + 1);
  DVec<int> tot(1);
  if (n > 0) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, 0, cnt.p, ptr.p, n, tot.p);
    OKCHK();
  } else {
    OCHK(hipMemset(tot.p, 0, sizeof(int)));
  }
  OCHK(hipMemcpy(ptr.p + n, tot.p, sizeof(int), hipMemcpyDeviceToDevice));
  int t = 0;
  OCHK(hipMemcpy(&t, tot.p, sizeof(int), hipMemcpyDeviceToHost));
  return t;
}

// unique values of a sorted key array
int64_t unique_sorted(const DVec<uint64_t>& a, int64_t n, DVec<uint64_t>& out) {
  DVec<int> flag(std::max<int64_t>(n, 1)), pos;
  hipLaunchKernelGGL(k_heads, grid_for(n), dim3(256), 0, 0, a.p, n, flag.p);
  OKCHK();
  const int m = scan_counts(flag, n, pos);
  out.alloc(std::max(m, 1));
  hipLaunchKernelGGL(k_compact, grid_for(n), dim3(256), 0, 0, a.p, n, flag.p, pos.p, out.p);
  OKCHK();
  return m;
}

}  // namespace

void Octree::build_device(const double* tgt, int64_t nt, const double* src, int64_t ns, int leaf_src,
                          double min_leaf_side, int depth_req) {
  if (nt < 1 || ns < 1) fail(LB_EINVAL, "octree: empty point set");
  if (nt >= (1ll << 31) || ns >= (1ll << 31)) fail(LB_EINVAL, "octree: more than 2^31 points");
  DVec<double> dt(3 * nt), ds(3 * ns);
  OCHK(hipMemcpy(dt.p, tgt, sizeof(double) * 3 * nt, hipMemcpyHostToDevice));
  OCHK(hipMemcpy(ds.p, src, sizeof(double) * 3 * ns, hipMemcpyHostToDevice));
  // frame
  const int nmm = (int)std::min<int64_t>(1024, (nt + ns + 255) / 256);
  DVec<double> part((size_t)nmm * 6);
  hipLaunchKernelGGL(k_minmax, dim3(nmm), dim3(256), 0, 0, dt.p, nt, ds.p, ns, part.p);
  OKCHK();
  std::vector<double> ph = part.host((size_t)nmm * 6);
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (int b = 0; b < nmm; ++b)
    for (int d = 0; d < 3; ++d) {
      mn[d] = std::min(mn[d], ph[6 * b + d]);
      mx[d] = std::max(mx[d], ph[6 * b + 3 + d]);
    }
  set_frame(mn, mx);
  const double scale = (double)(1 << 21) / side;
  DVec<uint64_t> kt(nt), ks(ns);
  hipLaunchKernelGGL(k_keys, grid_for(nt), dim3(256), 0, 0, dt.p, nt, lo[0], lo[1], lo[2], scale, kt.p);
  OKCHK();
  hipLaunchKernelGGL(k_keys, grid_for(ns), dim3(256), 0, 0, ds.p, ns, lo[0], lo[1], lo[2], scale, ks.p);
  OKCHK();
  // depth
  if (depth_req >= 0) {
    depth = std::min(depth_req, 20);
  } else {
    DVec<uint64_t> sk(ns);
    DVec<int> sv(ns);
    OCHK(hipMemcpy(sk.p, ks.p, sizeof(uint64_t) * ns, hipMemcpyDeviceToDevice));
    hipLaunchKernelGGL(k_iota, grid_for(ns), dim3(256), 0, 0, sv.p, ns);
    OKCHK();
    radix_sort(sk, sv, ns, 63);
    const int nb = (int)((ns + 255) / 256);
    DVec<int> pc((size_t)nb * 21);
    hipLaunchKernelGGL(k_level_counts, dim3(nb), dim3(256), 0, 0, sk.p, ns, pc.p);
    OKCHK();
    std::vector<int> h = pc.host((size_t)nb * 21);
    int64_t cnt[21] = {0};
    for (int b = 0; b < nb; ++b)
      for (int l = 2; l <= 20; ++l) cnt[l] += h[(size_t)b * 21 + l];
    depth = choose_depth(cnt, ns, leaf_src, min_leaf_side);
  }
  const int shift = 3 * (21 - depth);
  // stable orders by leaf key
  DVec<uint64_t> lt(nt), ls(ns);
  DVec<int> pt(nt), ps(ns);
  hipLaunchKernelGGL(k_shift, grid_for(nt), dim3(256), 0, 0, kt.p, nt, shift, lt.p);
  OKCHK();
  hipLaunchKernelGGL(k_shift, grid_for(ns), dim3(256), 0, 0, ks.p, ns, shift, ls.p);
  OKCHK();
  hipLaunchKernelGGL(k_iota, grid_for(nt), dim3(256), 0, 0, pt.p, nt);
  OKCHK();
  hipLaunchKernelGGL(k_iota, grid_for(ns), dim3(256), 0, 0, ps.p, ns);
  OKCHK();
  radix_sort(lt, pt, nt, 3 * depth);
  radix_sort(ls, ps, ns, 3 * depth);
  // unique leaf keys of both sets, then each coarser level from the finer one
  std::vector<DVec<uint64_t>> lk(depth + 1);
  std::vector<int64_t> nl(depth + 1);
  {
    DVec<uint64_t> all(nt + ns);
    DVec<int> av(nt + ns);
    OCHK(hipMemcpy(all.p, lt.p, sizeof(uint64_t) * nt, hipMemcpyDeviceToDevice));
    OCHK(hipMemcpy(all.p + nt, ls.p, sizeof(uint64_t) * ns, hipMemcpyDeviceToDevice));
    hipLaunchKernelGGL(k_iota, grid_for(nt + ns), dim3(256), 0, 0, av.p, nt + ns);
    OKCHK();
    radix_sort(all, av, nt + ns, 3 * depth);
    nl[depth] = unique_sorted(all, nt + ns, lk[depth]);
  }
  for (int l = depth - 1; l >= 0; --l) {
    DVec<uint64_t> pk(nl[l + 1]);
    hipLaunchKernelGGL(k_shift, grid_for(nl[l + 1]), dim3(256), 0, 0, lk[l + 1].p, nl[l + 1], 3, pk.p);
    OKCHK();
    nl[l] = unique_sorted(pk, nl[l + 1], lk[l]);
  }
  lev_off.assign(depth + 2, 0);
  for (int l = 0; l <= depth; ++l) lev_off[l + 1] = lev_off[l] + (int)nl[l];
  const int nb = lev_off[depth + 1];
  const int nleaf = (int)nl[depth];
  DVec<uint64_t> keys(nb);
  for (int l = 0; l <= depth; ++l)
    OCHK(hipMemcpy(keys.p + lev_off[l], lk[l].p, sizeof(uint64_t) * nl[l], hipMemcpyDeviceToDevice));
  DVec<int> loff(depth + 2);
  OCHK(hipMemcpy(loff.p, lev_off.data(), sizeof(int) * (depth + 2), hipMemcpyHostToDevice));
  DVec<int> dbx(nb), dby(nb), dbz(nb), dpar(nb), dch((size_t)nb * 8);
  OCHK(hipMemset(dch.p, 0xff, sizeof(int) * (size_t)nb * 8));
  hipLaunchKernelGGL(k_boxes, grid_for(nb), dim3(256), 0, 0, keys.p, loff.p, depth, nb, dbx.p, dby.p, dbz.p,
                     dpar.p, dch.p);
  OKCHK();
  DVec<unsigned char> dhs(nb), dht(nb);
  OCHK(hipMemset(dhs.p, 0, nb));
  OCHK(hipMemset(dht.p, 0, nb));
  DVec<int> tb(nleaf), te(nleaf), sb(nleaf), se(nleaf);
  hipLaunchKernelGGL(k_leaf_ranges, grid_for(nleaf), dim3(256), 0, 0, lk[depth].p, nleaf, lt.p, nt, ls.p, ns, tb.p,
                     te.p, sb.p, se.p, dhs.p, dht.p, lev_off[depth]);
  OKCHK();
  for (int l = depth - 1; l >= 0; --l) {
    hipLaunchKernelGGL(k_has_up, grid_for(lev_off[l + 1] - lev_off[l]), dim3(256), 0, 0, dch.p, lev_off[l],
                       lev_off[l + 1], dhs.p, dht.p);
    OKCHK();
  }
  // U-lists and V-lists: count, scan, fill
  DVec<int> ucnt(std::max(nleaf, 1)), uptr, ul;
  hipLaunchKernelGGL(k_ulist<false>, grid_for(nleaf), dim3(256), 0, 0, keys.p, loff.p, depth, nleaf, dbx.p, dby.p,
                     dbz.p, dhs.p, dht.p, ucnt.p, nullptr, nullptr);
  OKCHK();
  const int nu = scan_counts(ucnt, nleaf, uptr);
  ul.alloc(std::max(nu, 1));
  hipLaunchKernelGGL(k_ulist<true>, grid_for(nleaf), dim3(256), 0, 0, keys.p, loff.p, depth, nleaf, dbx.p, dby.p,
                     dbz.p, dhs.p, dht.p, nullptr, uptr.p, ul.p);
  OKCHK();
  DVec<int> vcnt(std::max(nb, 1)), vptr, vs, vo;
  hipLaunchKernelGGL(k_vlist<false>, grid_for(nb), dim3(256), 0, 0, keys.p, loff.p, nb, dbx.p, dby.p, dbz.p, dpar.p,
                     dch.p, dhs.p, dht.p, vcnt.p, nullptr, nullptr, nullptr);
  OKCHK();
  const int nv = scan_counts(vcnt, nb, vptr);
  vs.alloc(std::max(nv, 1));
  vo.alloc(std::max(nv, 1));
  hipLaunchKernelGGL(k_vlist<true>, grid_for(nb), dim3(256), 0, 0, keys.p, loff.p, nb, dbx.p, dby.p, dbz.p, dpar.p,
                     dch.p, dhs.p, dht.p, nullptr, vptr.p, vs.p, vo.p);
  OKCHK();
  OCHK(hipDeviceSynchronize());
  // results to the host structure
  bx = dbx.host(nb); by = dby.host(nb); bz = dbz.host(nb);
  parent = dpar.host(nb);
  child = dch.host((size_t)nb * 8);
  has_src = dhs.host(nb);
  has_tgt = dht.host(nb);
  tgt_beg = tb.host(nleaf); tgt_end = te.host(nleaf);
  src_beg = sb.host(nleaf); src_end = se.host(nleaf);
  ulist_ptr = uptr.host(nleaf + 1);
  ulist = ul.host(nu);
  vlist_ptr = vptr.host(nb + 1);
  vlist_src = vs.host(nv);
  vlist_off = vo.host(nv);
  std::vector<int> hpt = pt.host(nt), hps = ps.host(ns);
  tgt_perm.assign(hpt.begin(), hpt.end());
  src_perm.assign(hps.begin(), hps.end());
  tgt_pos.resize(nt);
  src_pos.resize(ns);
  for (int64_t j = 0; j < nt; ++j) tgt_pos[tgt_perm[j]] = j;
  for (int64_t j = 0; j < ns; ++j) src_pos[src_perm[j]] = j;
  max_leaf_tgt = max_leaf_src = 0;
  for (int b = 0; b < nleaf; ++b) {
    max_leaf_tgt = std::max(max_leaf_tgt, tgt_end[b] - tgt_beg[b]);
    max_leaf_src = std::max(max_leaf_src, src_end[b] - src_beg[b]);
  }
}

}  // namespace lb
