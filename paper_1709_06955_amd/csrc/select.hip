// Output selection of a finished query: the top-k of Definition 2 (k nodes
// v != u of largest estimate, ties to the smaller id, in that order) and the
// ascending list of nonzero estimates.
//
// Top-k is a radix select over the estimates, most significant digit first:
// each pass histograms, in LDS, the next digit of every estimate whose higher
// digits equal the prefix chosen so far, and the last workgroup to finish
// picks the digit that holds the k-th largest key.  The select stops as soon
// as that digit's bucket holds exactly the keys still needed (usually after
// one or two passes), or when all 64 bits are fixed (the remaining keys are
// equal and the smaller ids win).  One pass then collects the keys above the
// bucket and, in id order, the needed keys of the bucket; an LDS bitonic sort
// of the k (key, id) pairs orders them.  Every pass reads the n estimates
// once (8 bytes per node) and writes nothing of size n.
//
// The nonzero list is an ordered compaction: per-workgroup counts over
// contiguous id ranges, then each workgroup writes its entries at the offset
// the counts before it give.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "ps_internal.h"

namespace {

constexpr int kSelBlock = 256;
constexpr int kSelMaxGrid = 2048;
constexpr int kSelHist = 8192;    // buckets of the widest digit (13 bits)
constexpr int kSortTile = 4096;   // pairs one workgroup sorts in LDS
constexpr int kSortThreads = 1024;
constexpr int kPasses = 5;
// digit widths, most significant first: sign and exponent, then the mantissa
constexpr int kDigitBits[kPasses] = {12, 13, 13, 13, 13};

struct SelState {
  unsigned long long pre;  // the fixed high bits of the bucket of the k-th key
  int32_t sh;              // bits below the fixed ones
  int32_t need;            // keys of that bucket that belong to the top-k
  int32_t exact;           // the bucket holds exactly `need` keys
  uint32_t ticket;         // workgroups done with the current pass
  uint32_t n_gt;           // keys above the bucket collected so far
  uint32_t n_eq;           // keys of the bucket collected so far (exact case)
  unsigned long long total;  // nonzero count (compaction)
  uint32_t hist[kSelHist];
  uint32_t cnt[kSelMaxGrid];  // per-workgroup counts (ordered compaction)
};

// Order-preserving map of a double to an unsigned key (larger value, larger
// key; -0 and +0 map to the same key).
__device__ inline unsigned long long okey(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x + 0.0);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// `before(a, b)`: a ranks ahead of b (larger key, then smaller id).
__device__ inline bool before(unsigned long long ka, int32_t ia, unsigned long long kb, int32_t ib) {
  return ka > kb || (ka == kb && ia < ib);
}

__device__ inline void range_of(int32_t n, int64_t* lo, int64_t* hi) {
  const int64_t per = ((int64_t)n + gridDim.x - 1) / gridDim.x;
  *lo = std::min<int64_t>((int64_t)blockIdx.x * per, n);
  *hi = std::min<int64_t>(*lo + per, n);
}

// Exclusive prefix sum over the workgroup; returns the workgroup total.
__device__ uint32_t wg_excl_scan(uint32_t x, uint32_t* excl, uint32_t* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) lds[wave] = incl;
  __syncthreads();
  uint32_t before_w = 0, total = 0;
  for (int w = 0; w < nw; ++w) {
    const uint32_t s = lds[w];
    if (w < wave) before_w += s;
    total += s;
  }
  __syncthreads();
  *excl = before_w + incl - x;
  return total;
}

__global__ void k_sel_init(SelState* st, int32_t k) {
  for (int i = threadIdx.x; i < kSelHist; i += blockDim.x) st->hist[i] = 0;
  if (threadIdx.x == 0) {
    st->pre = 0;
    st->sh = 64;
    st->need = k;
    st->exact = 0;
    st->ticket = 0;
    st->n_gt = 0;
    st->n_eq = 0;
    st->total = 0;
  }
}

// One radix pass: histogram of the next digit of the keys in the current
// bucket; the last workgroup picks the bucket of the k-th key.
__global__ void __launch_bounds__(kSelBlock) k_sel_pass(int32_t n, int32_t u, const double* __restrict__ s,
                                                       SelState* st, int bits) {
  __shared__ uint32_t h[kSelHist];
  __shared__ uint32_t scan[kSelBlock];
  __shared__ int last;
  if (st->exact || st->sh == 0) return;  // uniform: the select already ended
  const int sh_old = st->sh, sh_new = sh_old - bits;
  const unsigned long long pre = st->pre;
  const int nb = 1 << bits;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) h[i] = 0;
  __syncthreads();
  int64_t lo, hi;
  range_of(n, &lo, &hi);
  for (int64_t v = lo + threadIdx.x; v < hi; v += blockDim.x) {
    if (v == u) continue;
    const unsigned long long key = okey(s[v]);
    if (sh_old < 64 && (key >> sh_old) != pre) continue;
    atomicAdd(&h[(uint32_t)(key >> sh_new) & (uint32_t)(nb - 1)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
    if (h[i]) atomicAdd(&st->hist[i], h[i]);
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(&st->ticket, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  // suffix sums over the buckets, from the top digit down
  const int per = nb / kSelBlock;
  const int b0 = threadIdx.x * per;
  uint32_t mine = 0;
  for (int i = 0; i < per; ++i) {
    h[b0 + i] = __hip_atomic_load(&st->hist[b0 + i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    mine += h[b0 + i];
  }
  scan[threadIdx.x] = mine;
  __syncthreads();
  for (int d = 1; d < kSelBlock; d <<= 1) {
    const uint32_t y = threadIdx.x + d < kSelBlock ? scan[threadIdx.x + d] : 0;
    __syncthreads();
    scan[threadIdx.x] += y;
    __syncthreads();
  }
  const uint32_t need = (uint32_t)st->need;
  const uint32_t suf = scan[threadIdx.x], above0 = suf - mine;
  __syncthreads();
  if (above0 < need && suf >= need) {  // exactly one thread holds the crossing
    uint32_t above = above0;
    for (int i = per - 1; i >= 0; --i) {
      const uint32_t c = h[b0 + i];
      if (above + c >= need) {
        st->pre = (sh_old == 64 ? 0ull : pre << bits) | (unsigned long long)(b0 + i);
        st->sh = sh_new;
        st->need = (int32_t)(need - above);
        st->exact = c == need - above;
        break;
      }
      above += c;
    }
  }
  for (int i = threadIdx.x; i < nb; i += blockDim.x) st->hist[i] = 0;
  if (threadIdx.x == 0) st->ticket = 0;
}

// Predicates of the collection pass: 2 = above the bucket, 1 = in it.
__device__ inline int bucket_of(unsigned long long key, unsigned long long pre, int sh) {
  const unsigned long long hiw = sh >= 64 ? 0ull : key >> sh;
  return hiw > pre ? 2 : (hiw == pre ? 1 : 0);
}

// Per-workgroup count of the keys in the bucket (only when it holds more
// keys than needed and the smaller ids must be taken).
__global__ void __launch_bounds__(kSelBlock) k_sel_count(int32_t n, int32_t u, const double* __restrict__ s,
                                                        SelState* st) {
  __shared__ uint32_t lds[kSelBlock / 64];
  if (st->exact) return;
  const unsigned long long pre = st->pre;
  const int sh = st->sh;
  int64_t lo, hi;
  range_of(n, &lo, &hi);
  uint32_t c = 0;
  for (int64_t v = lo + threadIdx.x; v < hi; v += blockDim.x)
    c += v != u && bucket_of(okey(s[v]), pre, sh) == 1;
  uint32_t ex;
  const uint32_t tot = wg_excl_scan(c, &ex, lds);
  if (threadIdx.x == 0) st->cnt[blockIdx.x] = tot;
}

// Collects the k selected (key, id) pairs: the keys above the bucket first
// (any order), then the needed keys of the bucket.
__global__ void __launch_bounds__(kSelBlock) k_sel_collect(int32_t n, int32_t u, const double* __restrict__ s,
                                                          SelState* st, int32_t k, unsigned long long* __restrict__ keys,
                                                          int32_t* __restrict__ ids) {
  __shared__ uint32_t lds[kSelBlock / 64];
  __shared__ uint32_t base_s;
  const unsigned long long pre = st->pre;
  const int sh = st->sh;
  const uint32_t need = (uint32_t)st->need, n_gt_all = (uint32_t)k - need;
  const bool exact = st->exact != 0;
  int64_t lo, hi;
  range_of(n, &lo, &hi);
  if (!exact) {
    uint32_t c = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += blockDim.x) c += st->cnt[b];
    uint32_t ex;
    const uint32_t tot = wg_excl_scan(c, &ex, lds);
    if (threadIdx.x == 0) base_s = tot;
    __syncthreads();
  }
  uint32_t base = exact ? 0 : base_s;
  for (int64_t t0 = lo; t0 < hi; t0 += blockDim.x) {
    const int64_t v = t0 + threadIdx.x;
    int b = 0;
    unsigned long long key = 0;
    if (v < hi && v != u) {
      key = okey(s[v]);
      b = bucket_of(key, pre, sh);
    }
    if (b == 2) {
      const uint32_t at = atomicAdd(&st->n_gt, 1u);
      if (at < n_gt_all) {  // always, by the counts of the passes
        keys[at] = key;
        ids[at] = (int32_t)v;
      }
    }
    if (exact) {
      if (b == 1) {
        const uint32_t at = n_gt_all + atomicAdd(&st->n_eq, 1u);
        if (at < (uint32_t)k) {
          keys[at] = key;
          ids[at] = (int32_t)v;
        }
      }
    } else {
      if (base >= need) continue;  // uniform across the workgroup
      uint32_t ex;
      const uint32_t tot = wg_excl_scan(b == 1, &ex, lds);
      if (b == 1 && base + ex < need) {
        keys[n_gt_all + base + ex] = key;
        ids[n_gt_all + base + ex] = (int32_t)v;
      }
      base += tot;
    }
  }
}

// Bitonic sort into `before` order over a power-of-two count of pairs.
// `k_sort_tile` runs, inside one workgroup's tile of `tile` pairs (at most
// kSortTile), every stage up to the tile's width (size 0) or the strides
// below the tile width of a wider stage `size`; `k_sort_step` runs one
// global compare-exchange step of a wider stage.
__device__ inline void cmp_swap(unsigned long long* K, int32_t* I, int64_t i, int64_t j, bool up) {
  const unsigned long long ka = K[i], kb = K[j];
  const int32_t ia = I[i], ib = I[j];
  if (up ? before(kb, ib, ka, ia) : before(ka, ia, kb, ib)) {
    K[i] = kb;
    K[j] = ka;
    I[i] = ib;
    I[j] = ia;
  }
}

__global__ void __launch_bounds__(kSortThreads) k_sort_tile(unsigned long long* __restrict__ keys,
                                                           int32_t* __restrict__ ids, int tile, int64_t size) {
  __shared__ unsigned long long K[kSortTile];
  __shared__ int32_t I[kSortTile];
  const int64_t t0 = (int64_t)blockIdx.x * tile;
  for (int i = threadIdx.x; i < tile; i += blockDim.x) {
    K[i] = keys[t0 + i];
    I[i] = ids[t0 + i];
  }
  __syncthreads();
  const int64_t s_lo = size ? size : 2, s_hi = size ? size : tile;
  for (int64_t sz = s_lo; sz <= s_hi; sz <<= 1) {
    for (int64_t st = std::min<int64_t>(sz, tile) >> 1; st > 0; st >>= 1) {
      for (int p = threadIdx.x; p < tile / 2; p += blockDim.x) {
        const int i = (int)((p / st) * 2 * st + p % st);
        cmp_swap(K, I, i, i + (int)st, ((t0 + i) & sz) == 0);
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < tile; i += blockDim.x) {
    keys[t0 + i] = K[i];
    ids[t0 + i] = I[i];
  }
}

__global__ void k_sort_step(unsigned long long* __restrict__ keys, int32_t* __restrict__ ids, int64_t total,
                            int64_t size, int64_t stride) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total / 2;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = (p / stride) * 2 * stride + p % stride;
    cmp_swap(keys, ids, i, i + stride, (i & size) == 0);
  }
}

__global__ void k_sort_pad(unsigned long long* __restrict__ keys, int32_t* __restrict__ ids, int64_t from,
                           int64_t to) {
  for (int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < to; i += (int64_t)gridDim.x * blockDim.x) {
    keys[i] = 0;  // below every estimate's key
    ids[i] = 0x7FFFFFFF;
  }
}

__global__ void k_sel_emit(const double* __restrict__ s, int32_t n, const int32_t* __restrict__ ids, int64_t k,
                           int32_t* __restrict__ out_ids, double* __restrict__ out_s) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = ids[i];
    const bool ok = v >= 0 && v < n;  // a pad entry here would mean a lost key
    out_ids[i] = ok ? v : -1;
    out_s[i] = ok ? s[v] : __longlong_as_double(0x7FF8000000000000ll);
  }
}

// Ordered compaction of the nonzero estimates: counts, then writes.
__global__ void __launch_bounds__(kSelBlock) k_nz_count(int32_t n, const double* __restrict__ s, SelState* st) {
  __shared__ uint32_t lds[kSelBlock / 64];
  int64_t lo, hi;
  range_of(n, &lo, &hi);
  uint32_t c = 0;
  for (int64_t v = lo + threadIdx.x; v < hi; v += blockDim.x) c += s[v] != 0.0;
  uint32_t ex;
  const uint32_t tot = wg_excl_scan(c, &ex, lds);
  if (threadIdx.x == 0) st->cnt[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kSelBlock) k_nz_write(int32_t n, const double* __restrict__ s, SelState* st,
                                                       int64_t cap, int32_t* __restrict__ out_ids,
                                                       double* __restrict__ out_s) {
  __shared__ uint32_t lds[kSelBlock / 64];
  int64_t lo, hi;
  range_of(n, &lo, &hi);
  uint32_t c = 0;
  for (uint32_t b = threadIdx.x; b < blockIdx.x; b += blockDim.x) c += st->cnt[b];
  uint32_t ex;
  uint64_t base = wg_excl_scan(c, &ex, lds);
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) st->total = base + st->cnt[blockIdx.x];
  for (int64_t t0 = lo; t0 < hi && (int64_t)base < cap; t0 += blockDim.x) {
    const int64_t v = t0 + threadIdx.x;
    const double x = v < hi ? s[v] : 0.0;
    const uint32_t tot = wg_excl_scan(x != 0.0, &ex, lds);
    if (x != 0.0 && (int64_t)(base + ex) < cap) {
      out_ids[base + ex] = (int32_t)v;
      out_s[base + ex] = x;
    }
    base += tot;
  }
}

int sel_grid(int32_t n) {
  const int64_t g = ((int64_t)n + kSelBlock * 8 - 1) / (kSelBlock * 8);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, kSelMaxGrid));
}

}  // namespace

namespace {

// The selection on caller-provided scratch: S (one SelState), K and I (room
// for `padded` pairs each, padded = the power of two >= max(k, 64)).
ps_status select_topk_on(SelState* S, unsigned long long* K, int32_t* I, int64_t padded, const double* s, int32_t n,
                         int32_t u, int32_t k, int32_t* out_ids, double* out_s, hipStream_t st) {
  const int tile = (int)std::min<int64_t>(padded, kSortTile);
  const int grid = sel_grid(n);
  k_sel_init<<<1, kSelBlock, 0, st>>>(S, k);
  for (int p = 0; p < kPasses; ++p) k_sel_pass<<<grid, kSelBlock, 0, st>>>(n, u, s, S, kDigitBits[p]);
  k_sel_count<<<grid, kSelBlock, 0, st>>>(n, u, s, S);
  k_sort_pad<<<(int)std::min<int64_t>((padded + kSelBlock - 1) / kSelBlock, 1024), kSelBlock, 0, st>>>(K, I, 0,
                                                                                                  padded);
  k_sel_collect<<<grid, kSelBlock, 0, st>>>(n, u, s, S, k, K, I);
  const int tiles = (int)(padded / tile);
  const int threads = std::min(kSortThreads, std::max(64, tile / 2));
  k_sort_tile<<<tiles, threads, 0, st>>>(K, I, tile, 0);
  for (int64_t size = 2 * kSortTile; size <= padded; size <<= 1) {
    for (int64_t stride = size / 2; stride >= kSortTile; stride >>= 1) {
      const int64_t pairs = padded / 2;
      const int g = (int)std::min<int64_t>((pairs + kSelBlock - 1) / kSelBlock, 4096);
      k_sort_step<<<g, kSelBlock, 0, st>>>(K, I, padded, size, stride);
    }
    k_sort_tile<<<tiles, threads, 0, st>>>(K, I, tile, size);
  }
  k_sel_emit<<<(int)std::min<int64_t>((k + kSelBlock - 1) / kSelBlock, 4096), kSelBlock, 0, st>>>(s, n, I, k, out_ids,
                                                                                                 out_s);
  PS_HIP(hipGetLastError());
  return PS_OK;
}

int64_t padded_for(int32_t k) {
  int64_t padded = 64;
  while (padded < k) padded <<= 1;
  return padded;
}

}  // namespace

ps_status select_topk(SelectBufs& b, const double* s, int32_t n, int32_t u, int32_t k, int32_t* out_ids,
                      double* out_s, hipStream_t st) {
  if (k < 1 || k > n - 1) return PS_ERR_INVALID_ARG;
  TraceRange tr("probesim top-k selection");
  const int64_t padded = padded_for(k);
  PS_TRY(devbuf_reserve(b.state, sizeof(SelState)));
  PS_TRY(devbuf_reserve(b.keys, sizeof(unsigned long long) * (size_t)padded));
  PS_TRY(devbuf_reserve(b.ids, sizeof(int32_t) * (size_t)padded));
  return select_topk_on(b.state.as<SelState>(), b.keys.as<unsigned long long>(), b.ids.as<int32_t>(), padded, s, n,
                        u, k, out_ids, out_s, st);
}

ps_status select_nonzero(SelectBufs& b, const double* s, int32_t n, int64_t cap, int32_t* out_ids, double* out_s,
                         int64_t* total, hipStream_t st) {
  PS_TRY(devbuf_reserve(b.state, sizeof(SelState)));
  SelState* S = b.state.as<SelState>();
  const int grid = sel_grid(n);
  k_nz_count<<<grid, kSelBlock, 0, st>>>(n, s, S);
  k_nz_write<<<grid, kSelBlock, 0, st>>>(n, s, S, cap, out_ids, out_s);
  PS_HIP(hipGetLastError());
  PS_HIP(hipMemcpyAsync(&b.h_total, &S->total, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  PS_HIP(hipStreamSynchronize(st));
  *total = (int64_t)b.h_total;
  return PS_OK;
}

// ------------------------------------------------- allocation-free variant --
//
// ps_select_topk_noalloc keeps its scratch (one SelState and room for
// kNoAllocMaxK (key, id) pairs) in the file-scope array below: one copy per
// device, held until the process ends.  In host code `scratch` names a host
// stand-in, never the device memory: its device address is looked up once
// per device (select_scratch_init, from ps_ctx_create with the device
// current) and only that address reaches kernels.

namespace {

constexpr size_t kStateBytes = (sizeof(SelState) + 255) & ~(size_t)255;
constexpr size_t kNoAllocBytes = kStateBytes + (size_t)PS_NOALLOC_MAX_K * (sizeof(unsigned long long) + sizeof(int32_t));
static_assert((PS_NOALLOC_MAX_K & (PS_NOALLOC_MAX_K - 1)) == 0, "the pair room must be a power of two");

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

ps_status select_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return PS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return PS_OK;
  void* p = nullptr;
  PS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) return PS_ERR_DEVICE;
  g_scratch[device] = p;
  return PS_OK;
}

extern "C" ps_status ps_select_topk_noalloc(ps_ctx* c, const double* s, int32_t n, int32_t u, int32_t k,
                                            int32_t* nodes, double* out_scores) {
  if (!c || !s || !nodes || !out_scores || n < 2) return PS_ERR_INVALID_ARG;
  if (u < 0 || u >= n) return PS_ERR_NODE_RANGE;
  if (k < 1 || k > n - 1 || k > PS_NOALLOC_MAX_K) return PS_ERR_INVALID_ARG;
  if (!ps_is_device_ptr(s) || !ps_is_device_ptr(nodes) || !ps_is_device_ptr(out_scores)) return PS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(c->mu);
  PS_HIP(hipSetDevice(c->device));
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk2(g_scratch_mu);
    if (c->device < kMaxDevices) base = g_scratch[c->device];
  }
  if (!base) return PS_ERR_STATE;  // the context's set-up did not find the array
  auto* S = reinterpret_cast<SelState*>(base);
  auto* K = reinterpret_cast<unsigned long long*>(static_cast<unsigned char*>(base) + kStateBytes);
  auto* I = reinterpret_cast<int32_t*>(K + PS_NOALLOC_MAX_K);
  return select_topk_on(S, K, I, padded_for(k), s, n, u, k, nodes, out_scores, c->stream);
}
