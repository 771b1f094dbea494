// cache.hip -- out-of-core brick cache (Sec 4.2: a GPU cache of chunks that
// keeps as many as it can and drops the least recently used; Sec 5.2: blocks
// missing from the cache are requested and their parent rendered instead;
// Sec 5.4: time series streamed through the cache).
//
// The pool holds cache_slots bricks. The host mirrors the page table
// ((t, c, node) -> slot or -1) and the slot owners. Renders stamp the slots
// of the nodes they use with a frame number (cut-map kernel) and append
// missing children to a request list. A put that finds no free slot reads
// the stamps back and evicts the oldest slots through a min-heap, never a
// top-level node's (the traversal starts there). Bricks arrive whole (core
// and apron), so no neighbour is needed to store one.
#include <algorithm>
#include <functional>
#include <queue>
#include <vector>

#include "sg_internal.h"

namespace sg {

namespace {

// Copy n stored regions ((B+2)^3 voxels, x fastest) into their slots (rows
// padded to Sx).
template <typename T>
__global__ __launch_bounds__(256) void put_kernel(uint8_t* pool, int64_t slot_bytes,
                                                  const int32_t* slots, const T* src, int n,
                                                  int S, int Sx, int M) {
  const int64_t per = (int64_t)S * S * S;
  const int64_t total = per * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = i / per, r = i - b * per;
    const int64_t row = r / S, x = r - row * S;
    T* dst = reinterpret_cast<T*>(pool + (int64_t)slots[b] * slot_bytes);
    dst[slot_index((int)x, (int)(row % S), (int)(row / S), S, Sx, M)] = src[i];
  }
}

// page[idx[i]] = val[i]
__global__ void scatter_kernel(int32_t* page, const int32_t* idx, const int32_t* val, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    page[idx[i]] = val[i];
}

// range[entry] = (min, max) of the stored region of its slot, one workgroup
// per brick.
template <typename T>
__global__ __launch_bounds__(256) void range_list_kernel(const uint8_t* pool, int64_t slot_bytes,
                                                         const int32_t* slots,
                                                         const int32_t* entries,
                                                         uint32_t* range, int S, int Sx,
                                                         int M) {
  const T* p = reinterpret_cast<const T*>(pool + (int64_t)slots[blockIdx.x] * slot_bytes);
  const int32_t n = S * S * S;
  uint32_t lo = 0xFFFFFFFFu, hi = 0;
  for (int32_t i = threadIdx.x; i < n; i += 256) {
    const int32_t row = i / S, x = i - row * S;
    const uint32_t v = p[slot_index(x, row % S, row / S, S, Sx, M)];
    lo = min(lo, v);
    hi = max(hi, v);
  }
  __shared__ uint32_t slo[256], shi[256];
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      slo[threadIdx.x] = min(slo[threadIdx.x], slo[threadIdx.x + s]);
      shi[threadIdx.x] = max(shi[threadIdx.x], shi[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t e = entries[blockIdx.x];
    range[2 * e] = slo[0];
    range[2 * e + 1] = shi[0];
  }
}

// Clear the flag bits of the listed entries (the list holds every set bit
// unless it overflowed).
__global__ void clear_requests_kernel(uint32_t* flags, const uint32_t* list,
                                      const uint32_t* count, int cap) {
  const uint32_t n = min(*count, (uint32_t)cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t e = list[i];
    atomicAnd(flags + (e >> 5), ~(1u << (e & 31)));
  }
}

__global__ void clear_all_kernel(uint32_t* flags, int64_t words) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    flags[i] = 0u;
}

// A freshly stored brick counts as used now: stamp[slot[i]] = frame.
__global__ void stamp_kernel(uint32_t* stamp, const int32_t* slot, int n, uint32_t frame) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    stamp[slot[i]] = frame;
}

__global__ void zero_count_kernel(uint32_t* count) {
  if (threadIdx.x == 0) *count = 0u;
}

int64_t entry_of(const Volume* v, int t, int c, int64_t node) {
  return ((int64_t)t * v->d.channels + c) * v->nodes + node;
}

bool is_top(const Volume* v, int64_t entry) {
  const int64_t node = entry % v->nodes;
  return node >= v->node_off[v->L - 1];
}

}  // namespace

bool top_level_resident(const Volume* v, int t) {
  if (!v->cache) return true;
  for (int c = 0; c < v->d.channels; ++c)
    for (int64_t n = v->node_off[v->L - 1]; n < v->nodes; ++n)
      if (v->page_host[(size_t)entry_of(v, t, c, n)] < 0) return false;
  return true;
}

}  // namespace sg

using namespace sg;

namespace {

// Both put entry points: the regions come from one buffer (src, host or
// device) or from one pointer per brick (srcs, any memory; each copied by
// its own DMA into the staging buffer).
sg_status put_impl(sg_volume* vol, int32_t channel, int32_t timepoint, int32_t level, int32_t n,
                   const int32_t* coords, const void* src, const void* const* srcs,
                   int32_t src_on_device, void* hip_stream) {
  if (!vol) return fail(SG_ERR_INVALID_ARG, "sg_cache_put: NULL volume");
  Volume* v = &vol->v;
  if (!v->cache) return fail(SG_ERR_UNSUPPORTED, "sg_cache_put: not a cache volume");
  if (channel < 0 || channel >= v->d.channels || timepoint < 0 ||
      timepoint >= v->d.timepoints || level < 0 || level >= v->L || n < 0)
    return fail(SG_ERR_INVALID_ARG, "sg_cache_put: channel/timepoint/level/n out of range");
  if (n == 0) return SG_OK;
  if (!coords || (!src && !srcs))
    return fail(SG_ERR_INVALID_ARG, "sg_cache_put: NULL coords or source");
  if (srcs)
    for (int32_t i = 0; i < n; ++i)
      if (!srcs[i]) return fail(SG_ERR_INVALID_ARG, "sg_cache_put_scattered: NULL region pointer");
  std::vector<int64_t> ent((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    for (int a = 0; a < 3; ++a)
      if (coords[3 * i + a] < 0 || coords[3 * i + a] >= v->grid[level][a])
        return fail(SG_ERR_INVALID_ARG, "sg_cache_put: brick coordinate outside the grid");
    const int64_t node = v->node_off[level] +
                         ((int64_t)coords[3 * i + 2] * v->grid[level][1] + coords[3 * i + 1]) *
                             v->grid[level][0] +
                         coords[3 * i];
    ent[(size_t)i] = entry_of(v, timepoint, channel, node);
  }
  {
    std::vector<int64_t> sorted = ent;
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
      return fail(SG_ERR_INVALID_ARG, "sg_cache_put: a brick appears twice");
  }
  DeviceGuard guard(v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  hipStream_t s = (hipStream_t)hip_stream;

  // slots: the brick's own if resident, else a free one, else the oldest
  // evictable one (min-heap over the stamps of the last renders)
  int need = 0;
  for (int64_t e : ent)
    if (v->page_host[(size_t)e] < 0) ++need;
  std::vector<int32_t> slot((size_t)n, -1);
  std::vector<int32_t> pidx, pval;  // page updates
  if (need > (int)v->free_slots.size()) {
    SG_HIP(hipStreamSynchronize(s));
    std::vector<uint32_t> stamp((size_t)v->slots);
    SG_HIP(hipMemcpy(stamp.data(), v->stamp, (size_t)v->slots * 4, hipMemcpyDeviceToHost));
    std::vector<char> keep((size_t)v->entries, 0);
    for (int64_t e : ent) keep[(size_t)e] = 1;
    typedef std::pair<uint32_t, int32_t> Item;  // (stamp, slot): oldest first
    std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
    for (int64_t sl = 0; sl < v->slots; ++sl) {
      const int64_t e = v->owner[(size_t)sl];
      if (e < 0 || keep[(size_t)e] || is_top(v, e)) continue;
      heap.push(Item(stamp[(size_t)sl], (int32_t)sl));
    }
    if ((int64_t)heap.size() + (int64_t)v->free_slots.size() < need)
      return fail(SG_ERR_OUT_OF_MEMORY,
                  "sg_cache_put: more bricks than the cache can free (top-level nodes are "
                  "never evicted)");
    while (need > (int)v->free_slots.size()) {
      const int32_t sl = heap.top().second;
      heap.pop();
      const int64_t e = v->owner[(size_t)sl];
      v->page_host[(size_t)e] = -1;
      v->owner[(size_t)sl] = -1;
      pidx.push_back((int32_t)e);
      pval.push_back(-1);
      v->free_slots.push_back(sl);
      ++v->evictions;
    }
  }
  for (int32_t i = 0; i < n; ++i) {
    const int64_t e = ent[(size_t)i];
    int32_t sl = v->page_host[(size_t)e];
    if (sl < 0) {
      sl = v->free_slots.back();
      v->free_slots.pop_back();
      v->page_host[(size_t)e] = sl;
      v->owner[(size_t)sl] = e;
      pidx.push_back((int32_t)e);
      pval.push_back(sl);
    }
    slot[(size_t)i] = sl;
  }
  v->uploads += n;

  // device side: regions, page updates, ranges
  const int64_t S3 = (int64_t)v->S * v->S * v->S;
  const int64_t data_bytes = S3 * v->bpv * n;
  const int64_t meta = 4 * ((int64_t)2 * n + 2 * (int64_t)pidx.size());
  const int64_t meta_pad = ((meta + 255) / 256) * 256;
  const bool staged = srcs || !src_on_device;
  uint8_t* tmp = nullptr;
  SG_HIP(hipMallocAsync((void**)&tmp, (size_t)(meta_pad + (staged ? data_bytes : 0)), s));
  std::vector<int32_t> host_meta;
  host_meta.insert(host_meta.end(), slot.begin(), slot.end());
  for (int64_t e : ent) host_meta.push_back((int32_t)e);
  host_meta.insert(host_meta.end(), pidx.begin(), pidx.end());
  host_meta.insert(host_meta.end(), pval.begin(), pval.end());
  SG_HIP(hipMemcpyAsync(tmp, host_meta.data(), host_meta.size() * 4, hipMemcpyHostToDevice, s));
  const void* dsrc = src;
  if (srcs) {
    // one copy per run of regions that lie back to back in the source
    const size_t region = (size_t)(S3 * v->bpv);
    for (int32_t i = 0; i < n;) {
      int32_t j = i + 1;
      while (j < n && (const uint8_t*)srcs[j] == (const uint8_t*)srcs[j - 1] + region) ++j;
      SG_HIP(hipMemcpyAsync(tmp + meta_pad + region * (size_t)i, srcs[i],
                            region * (size_t)(j - i), hipMemcpyDefault, s));
      i = j;
    }
    dsrc = tmp + meta_pad;
  } else if (!src_on_device) {
    SG_HIP(hipMemcpyAsync(tmp + meta_pad, src, (size_t)data_bytes, hipMemcpyHostToDevice, s));
    dsrc = tmp + meta_pad;
  }
  SG_HIP(hipStreamSynchronize(s));  // host buffers consumed before returning
  const int32_t* d_slot = reinterpret_cast<const int32_t*>(tmp);
  const int32_t* d_ent = d_slot + n;
  const int32_t* d_pidx = d_ent + n;
  const int32_t* d_pval = d_pidx + pidx.size();
  const int64_t work = S3 * n;
  const int blocks = (int)std::min<int64_t>((work + 255) / 256, 65536);
  if (v->bpv == 1) {
    hipLaunchKernelGGL(put_kernel<uint8_t>, dim3(blocks), dim3(256), 0, s, v->pool,
                       v->slot_bytes, d_slot, (const uint8_t*)dsrc, n, v->S, v->Sx, v->M);
    hipLaunchKernelGGL(range_list_kernel<uint8_t>, dim3(n), dim3(256), 0, s, v->pool,
                       v->slot_bytes, d_slot, d_ent, v->range, v->S, v->Sx, v->M);
  } else {
    hipLaunchKernelGGL(put_kernel<uint16_t>, dim3(blocks), dim3(256), 0, s, v->pool,
                       v->slot_bytes, d_slot, (const uint16_t*)dsrc, n, v->S, v->Sx, v->M);
    hipLaunchKernelGGL(range_list_kernel<uint16_t>, dim3(n), dim3(256), 0, s, v->pool,
                       v->slot_bytes, d_slot, d_ent, v->range, v->S, v->Sx, v->M);
  }
  hipLaunchKernelGGL(stamp_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v->stamp,
                     d_slot, n, v->frame);
  SG_HIP(hipGetLastError());
  if (!pidx.empty()) {
    hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)((pidx.size() + 255) / 256)), dim3(256), 0,
                       s, v->page, d_pidx, d_pval, (int)pidx.size());
    SG_HIP(hipGetLastError());
  }
  SG_HIP(hipFreeAsync(tmp, s));
  v->empty_dirty = true;
  return SG_OK;
}

}  // namespace

extern "C" sg_status sg_cache_put(sg_volume* vol, int32_t channel, int32_t timepoint,
                                  int32_t level, int32_t n, const int32_t* coords,
                                  const void* src, int32_t src_on_device, void* hip_stream) {
  return put_impl(vol, channel, timepoint, level, n, coords, src, nullptr, src_on_device,
                  hip_stream);
}

extern "C" sg_status sg_cache_put_scattered(sg_volume* vol, int32_t channel, int32_t timepoint,
                                            int32_t level, int32_t n, const int32_t* coords,
                                            const void* const* srcs, void* hip_stream) {
  if (!srcs && n > 0) return fail(SG_ERR_INVALID_ARG, "sg_cache_put_scattered: NULL srcs");
  return put_impl(vol, channel, timepoint, level, n, coords, nullptr, srcs, 0, hip_stream);
}

extern "C" sg_status sg_cache_requests(sg_volume* vol, uint64_t* ids, int32_t* timepoints,
                                       int32_t* n, void* hip_stream) {
  if (!vol || !n || *n < 0 || (*n > 0 && (!ids || !timepoints)))
    return fail(SG_ERR_INVALID_ARG, "sg_cache_requests: NULL argument or negative capacity");
  Volume* v = &vol->v;
  if (!v->cache) return fail(SG_ERR_UNSUPPORTED, "sg_cache_requests: not a cache volume");
  DeviceGuard guard(v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  hipStream_t s = (hipStream_t)hip_stream;
  uint32_t count = 0;
  SG_HIP(hipMemcpyAsync(&count, v->req_count, 4, hipMemcpyDeviceToHost, s));
  SG_HIP(hipStreamSynchronize(s));
  const int32_t m = (int32_t)std::min<uint32_t>(count, (uint32_t)kReqCap);
  if (m > *n) {
    *n = m;
    return fail(SG_ERR_INVALID_ARG, "sg_cache_requests: capacity too small");
  }
  std::vector<uint32_t> list((size_t)std::max(m, 1));
  if (m > 0)
    SG_HIP(hipMemcpyAsync(list.data(), v->req_list, (size_t)m * 4, hipMemcpyDeviceToHost, s));
  const int64_t words = ((int64_t)v->d.timepoints * v->nodes + 31) / 32;
  if (count > (uint32_t)kReqCap) {
    // the list overflowed: some set bits are not listed, so clear them all
    hipLaunchKernelGGL(clear_all_kernel, dim3((unsigned)std::min<int64_t>((words + 255) / 256,
                                                                          65536)),
                       dim3(256), 0, s, v->req_flags, words);
  } else {
    hipLaunchKernelGGL(clear_requests_kernel, dim3((unsigned)std::max(1, (m + 255) / 256)),
                       dim3(256), 0, s, v->req_flags, v->req_list, v->req_count, kReqCap);
  }
  hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(64), 0, s, v->req_count);
  SG_HIP(hipGetLastError());
  SG_HIP(hipStreamSynchronize(s));
  std::vector<std::pair<int32_t, uint64_t>> out;
  for (int32_t i = 0; i < m; ++i) {
    const int64_t e = list[(size_t)i];
    const int32_t t = (int32_t)(e / v->nodes);
    const int64_t node = e - (int64_t)t * v->nodes;
    int L = 0;
    while (L + 1 < v->L && node >= v->node_off[L + 1]) ++L;
    const int64_t r = node - v->node_off[L];
    const int64_t x = r % v->grid[L][0], y = (r / v->grid[L][0]) % v->grid[L][1],
                  z = r / ((int64_t)v->grid[L][0] * v->grid[L][1]);
    out.emplace_back(t, ((uint64_t)L << 60) | ((uint64_t)x << 40) | ((uint64_t)y << 20) |
                            (uint64_t)z);
  }
  std::sort(out.begin(), out.end());
  for (int32_t i = 0; i < m; ++i) {
    timepoints[i] = out[(size_t)i].first;
    ids[i] = out[(size_t)i].second;
  }
  *n = m;
  return SG_OK;
}

extern "C" sg_status sg_cache_get_info(const sg_volume* vol, sg_cache_info* info) {
  if (!vol || !info) return fail(SG_ERR_INVALID_ARG, "sg_cache_get_info: NULL argument");
  const Volume* v = &vol->v;
  info->capacity = v->slots;
  info->resident = v->cache ? v->slots - (int64_t)v->free_slots.size() : v->slots;
  info->uploads = v->uploads;
  info->evictions = v->evictions;
  info->frame = v->frame;
  return SG_OK;
}

extern "C" sg_status sg_cache_resident(const sg_volume* vol, int32_t channel, int32_t timepoint,
                                       int32_t level, const int32_t b[3], int32_t* resident) {
  if (!vol || !b || !resident) return fail(SG_ERR_INVALID_ARG, "sg_cache_resident: NULL argument");
  const Volume* v = &vol->v;
  if (channel < 0 || channel >= v->d.channels || timepoint < 0 ||
      timepoint >= v->d.timepoints || level < 0 || level >= v->L)
    return fail(SG_ERR_INVALID_ARG, "sg_cache_resident: out of range");
  for (int a = 0; a < 3; ++a)
    if (b[a] < 0 || b[a] >= v->grid[level][a])
      return fail(SG_ERR_INVALID_ARG, "sg_cache_resident: brick outside the grid");
  if (!v->cache) {
    *resident = 1;
    return SG_OK;
  }
  const int64_t node =
      v->node_off[level] + ((int64_t)b[2] * v->grid[level][1] + b[1]) * v->grid[level][0] + b[0];
  *resident = v->page_host[(size_t)entry_of(v, timepoint, channel, node)] >= 0 ? 1 : 0;
  return SG_OK;
}
