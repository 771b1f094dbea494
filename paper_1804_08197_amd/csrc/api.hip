// api.hip -- C-ABI entry points for volume lifetime, uploads, pyramid,
// transfer functions and error reporting (see include/sg.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "sg_internal.h"

namespace sg {

namespace {
thread_local std::string g_last_error;
}

sg_status fail(sg_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

sg_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SG_ERR_OUT_OF_MEMORY;
  return SG_ERR_DEVICE;
}

DeviceGuard::DeviceGuard(int dev) {
  if (hipGetDevice(&prev) != hipSuccess) {
    prev = -1;
    return;
  }
  ok = hipSetDevice(dev) == hipSuccess;
}

DeviceGuard::~DeviceGuard() {
  if (prev >= 0) (void)hipSetDevice(prev);
}

sg_status stage_to_device(Volume* v, const void* host, int64_t bytes, void* dev,
                          hipStream_t stream) {
  if (bytes <= 0) return SG_OK;
  // the ring slot used Volume::kStageRing uploads ago is free once its copy ran
  const int k = v->stage_next;
  v->stage_next = (k + 1) % Volume::kStageRing;
  if (v->stage_pending[k]) {
    SG_HIP(hipEventSynchronize(v->stage_done[k]));
    v->stage_pending[k] = false;
  }
  if (bytes > v->stage_cap[k]) {
    if (v->stage_host[k]) SG_HIP(hipHostFree(v->stage_host[k]));
    v->stage_host[k] = nullptr;
    v->stage_cap[k] = 0;
    int64_t cap = std::max<int64_t>(bytes, 1 << 16);
    SG_HIP(hipHostMalloc((void**)&v->stage_host[k], (size_t)cap, hipHostMallocDefault));
    v->stage_cap[k] = cap;
  }
  std::memcpy(v->stage_host[k], host, (size_t)bytes);
  SG_HIP(hipMemcpyAsync(dev, v->stage_host[k], (size_t)bytes, hipMemcpyHostToDevice, stream));
  SG_HIP(hipEventRecord(v->stage_done[k], stream));
  v->stage_pending[k] = true;
  return SG_OK;
}

sg_status timing_mark(Volume* v, hipStream_t s) {
  hipEvent_t e;
  if (!v->ev_free.empty()) {
    e = v->ev_free.back();
    v->ev_free.pop_back();
  } else {
    SG_HIP(hipEventCreate(&e));
  }
  v->ev_rec.push_back(e);
  SG_HIP(hipEventRecord(e, s));
  return SG_OK;
}

namespace {

bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

void free_all(Volume* v) {
  hipFree(v->pool);
  hipFree(v->page);
  hipFree(v->range);
  hipFree(v->empty);
  hipFree(v->info);
  hipFree(v->tf);
  if (v->queue) hipFree(v->queue);
  if (v->stamp) hipFree(v->stamp);
  if (v->req_flags) hipFree(v->req_flags);
  if (v->req_list) hipFree(v->req_list);
  if (v->req_count) hipFree(v->req_count);
  hipFree(v->cutmap);
  hipFree(v->view_dev);
  hipFree(v->mb_bits);
  hipFree(v->counters);
  for (int k = 0; k < Volume::kStageRing; ++k) {
    if (v->stage_host[k]) hipHostFree(v->stage_host[k]);
    if (v->stage_done[k]) hipEventDestroy(v->stage_done[k]);
  }
  for (hipEvent_t e : v->ev_free) hipEventDestroy(e);
  for (hipEvent_t e : v->ev_rec) hipEventDestroy(e);
}

sg_status create(const sg_volume_desc* d, sg_volume** out) {
  if (!d || !out) return fail(SG_ERR_INVALID_ARG, "sg_volume_create: NULL argument");
  *out = nullptr;
  for (int a = 0; a < 3; ++a)
    if (d->dims[a] < 1 || d->dims[a] > (1 << 20))
      return fail(SG_ERR_INVALID_ARG, "dims must be in [1, 2^20]");
  if (d->channels < 1 || d->channels > kMaxChannels)
    return fail(SG_ERR_INVALID_ARG, "channels must be in [1, 4]");
  if (d->timepoints < 1) return fail(SG_ERR_INVALID_ARG, "timepoints must be >= 1");
  if (d->dtype != SG_U8 && d->dtype != SG_U16)
    return fail(SG_ERR_INVALID_ARG, "dtype must be SG_U8 or SG_U16");
  if (!pow2(d->brick) || d->brick < 2 || d->brick > 256)
    return fail(SG_ERR_INVALID_ARG, "brick must be a power of two in [2, 256]");
  if (d->levels < 1 || d->levels > kMaxLevels)
    return fail(SG_ERR_INVALID_ARG, "levels must be in [1, 16]");
  if (d->device < 0) return fail(SG_ERR_INVALID_ARG, "device must be >= 0");
  if (d->cache_slots < 0) return fail(SG_ERR_INVALID_ARG, "cache_slots must be >= 0");
  if (d->layout != SG_LAYOUT_LINEAR && d->layout != SG_LAYOUT_MICROBLOCK)
    return fail(SG_ERR_INVALID_ARG, "layout must be SG_LAYOUT_LINEAR or SG_LAYOUT_MICROBLOCK");

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return fail(SG_ERR_DEVICE, "no HIP device available");
  if (d->device >= ndev) return fail(SG_ERR_INVALID_ARG, "device ordinal out of range");
  DeviceGuard guard(d->device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");

  sg_volume* h = new (std::nothrow) sg_volume();
  if (!h) return fail(SG_ERR_OUT_OF_MEMORY, "host allocation failed");
  Volume* v = &h->v;
  v->d = *d;
  v->bpv = d->dtype == SG_U8 ? 1 : 2;
  v->B = d->brick;
  v->logB = 0;
  while ((1 << v->logB) < v->B) ++v->logB;
  v->S = v->B + 2;
  v->Sx = ((v->S * v->bpv + kRowAlignBytes - 1) / kRowAlignBytes) * kRowAlignBytes / v->bpv;
  v->L = d->levels;
  int64_t nodes = 0;
  for (int L = 0; L < v->L; ++L) {
    for (int a = 0; a < 3; ++a) {
      int64_t n = d->dims[a];
      for (int l = 0; l < L; ++l) n = (n + 1) / 2;
      v->ldims[L][a] = (int32_t)n;
      v->grid[L][a] = (int32_t)((n + v->B - 1) / v->B);
    }
    v->node_off[L] = nodes;
    nodes += (int64_t)v->grid[L][0] * v->grid[L][1] * v->grid[L][2];
  }
  v->node_off[v->L] = nodes;
  v->nodes = nodes;
  v->M = d->layout == SG_LAYOUT_MICROBLOCK ? (v->S + 3) / 4 : 0;
  const int64_t S3 = v->M ? (int64_t)v->M * v->M * v->M * 64 : (int64_t)v->S * v->S * v->Sx;
  v->slot_bytes = ((S3 * v->bpv + 64 + 255) / 256) * 256;
  v->entries = (int64_t)d->timepoints * d->channels * nodes;
  if (v->entries > 0x7FFFFFFF) {
    delete h;
    return fail(SG_ERR_INVALID_ARG, "too many (channel, timepoint, node) entries");
  }
  v->cache = d->cache_slots > 0;
  v->slots = v->cache ? std::min<int64_t>(d->cache_slots, v->entries) : v->entries;
  const int64_t pool_bytes = v->slots * v->slot_bytes;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && (uint64_t)pool_bytes > free_b) {
    delete h;
    return fail(SG_ERR_OUT_OF_MEMORY, "brick pool larger than free device memory");
  }
  auto alloc = [&](void** p, int64_t bytes) -> bool {
    if (hipMalloc(p, (size_t)std::max<int64_t>(bytes, 1)) != hipSuccess) return false;
    v->bytes += (uint64_t)bytes;
    return true;
  };
  const int64_t tf_bytes = (int64_t)kMaxChannels * (kMaxTfEntries + 1) * 16 + 2 * kMaxChannels * 8;
  bool ok = alloc((void**)&v->pool, pool_bytes) &&
            alloc((void**)&v->page, v->entries * 4) &&
            alloc((void**)&v->range, v->entries * 8) &&
            alloc((void**)&v->empty, (int64_t)d->timepoints * nodes) &&
            alloc((void**)&v->info, nodes * (int64_t)sizeof(NodeInfo)) &&
            alloc((void**)&v->tf, tf_bytes);
  if (!ok) {
    free_all(v);
    delete h;
    (void)hipGetLastError();
    return fail(SG_ERR_OUT_OF_MEMORY, "device allocation failed");
  }
  if (v->cache &&
      !(alloc((void**)&v->stamp, v->slots * 4) &&
        alloc((void**)&v->req_flags, (((int64_t)d->timepoints * nodes + 31) / 32) * 4) &&
        alloc((void**)&v->req_list, (int64_t)kReqCap * 4) && alloc((void**)&v->req_count, 4))) {
    free_all(v);
    delete h;
    (void)hipGetLastError();
    return fail(SG_ERR_OUT_OF_MEMORY, "device allocation failed (cache tables)");
  }
  for (int k = 0; k < Volume::kStageRing; ++k)
    if (hipEventCreateWithFlags(&v->stage_done[k], hipEventDisableTiming) != hipSuccess) {
      free_all(v);
      delete h;
      return fail(SG_ERR_DEVICE, "event creation failed");
    }
  // page table: every node resident with slot = (t * C + c) * nodes + node,
  // or (cache) nothing resident and every slot free
  std::vector<int32_t> page((size_t)v->entries);
  for (int64_t i = 0; i < v->entries; ++i) page[(size_t)i] = v->cache ? -1 : (int32_t)i;
  if (v->cache) {
    v->page_host = page;
    v->owner.assign((size_t)v->slots, -1);
    v->free_slots.resize((size_t)v->slots);
    for (int64_t i = 0; i < v->slots; ++i)
      v->free_slots[(size_t)i] = (int32_t)(v->slots - 1 - i);
  }
  std::vector<NodeInfo> info((size_t)nodes);
  for (int L = 0; L < v->L; ++L)
    for (int32_t z = 0; z < v->grid[L][2]; ++z)
      for (int32_t y = 0; y < v->grid[L][1]; ++y)
        for (int32_t x = 0; x < v->grid[L][0]; ++x) {
          NodeInfo& n = info[(size_t)(v->node_off[L] +
                                      ((int64_t)z * v->grid[L][1] + y) * v->grid[L][0] + x)];
          n.level = L;
          n.b[0] = x;
          n.b[1] = y;
          n.b[2] = z;
        }
  hipError_t e = hipMemset(v->pool, 0, (size_t)pool_bytes);
  if (e == hipSuccess) e = hipMemset(v->range, 0, (size_t)(v->entries * 8));
  if (e == hipSuccess) e = hipMemset(v->empty, 0, (size_t)(d->timepoints * nodes));
  if (e == hipSuccess)
    e = hipMemcpy(v->page, page.data(), (size_t)v->entries * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess && v->cache) e = hipMemset(v->stamp, 0, (size_t)v->slots * 4);
  if (e == hipSuccess && v->cache)
    e = hipMemset(v->req_flags, 0, (size_t)(((int64_t)d->timepoints * nodes + 31) / 32) * 4);
  if (e == hipSuccess && v->cache) e = hipMemset(v->req_count, 0, 4);
  if (e == hipSuccess)
    e = hipMemcpy(v->info, info.data(), (size_t)nodes * sizeof(NodeInfo), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_all(v);
    delete h;
    return hip_fail(e, "sg_volume_create: initialisation");
  }
  v->pending.assign((size_t)d->timepoints * d->channels, v->cache ? 0 : 1);
  *out = h;
  return SG_OK;
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" {

sg_status sg_volume_create(const sg_volume_desc* desc, sg_volume** out) {
  return create(desc, out);
}

sg_status sg_volume_destroy(sg_volume* vol) {
  if (!vol) return fail(SG_ERR_INVALID_ARG, "sg_volume_destroy: NULL volume");
  {
    DeviceGuard guard(vol->v.d.device);
    (void)hipDeviceSynchronize();
    free_all(&vol->v);
  }
  delete vol;
  return SG_OK;
}

sg_status sg_upload_bricks(sg_volume* vol, int32_t channel, int32_t timepoint, int32_t level,
                           int32_t n, const int32_t* coords, const void* src,
                           int32_t src_on_device, void* hip_stream) {
  if (!vol) return fail(SG_ERR_INVALID_ARG, "sg_upload_bricks: NULL volume");
  Volume* v = &vol->v;
  if (v->cache)
    return fail(SG_ERR_UNSUPPORTED, "sg_upload_bricks: a cache volume takes whole bricks "
                                    "(sg_cache_put)");
  if (channel < 0 || channel >= v->d.channels || timepoint < 0 ||
      timepoint >= v->d.timepoints || level < 0 || level >= v->L || n < 0)
    return fail(SG_ERR_INVALID_ARG, "sg_upload_bricks: channel/timepoint/level/n out of range");
  if (n == 0) return SG_OK;
  if (!coords || !src) return fail(SG_ERR_INVALID_ARG, "sg_upload_bricks: NULL coords or src");
  for (int32_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a)
      if (coords[3 * i + a] < 0 || coords[3 * i + a] >= v->grid[level][a])
        return fail(SG_ERR_INVALID_ARG, "sg_upload_bricks: brick coordinate outside the grid");
  DeviceGuard guard(v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t data_bytes = ((int64_t)n << (3 * v->logB)) * v->bpv;
  const int64_t coord_bytes = (int64_t)n * 3 * 4;
  uint8_t* tmp = nullptr;
  const int64_t tmp_bytes = ((coord_bytes + 255) / 256) * 256 + (src_on_device ? 0 : data_bytes);
  SG_HIP(hipMallocAsync((void**)&tmp, (size_t)tmp_bytes, s));
  const int64_t coff = src_on_device ? 0 : data_bytes;
  SG_HIP(hipMemcpyAsync(tmp + coff, coords, (size_t)coord_bytes, hipMemcpyHostToDevice, s));
  const void* dsrc = src;
  if (!src_on_device) {
    SG_HIP(hipMemcpyAsync(tmp, src, (size_t)data_bytes, hipMemcpyHostToDevice, s));
    dsrc = tmp;
  }
  // host buffers must be consumed before returning
  SG_HIP(hipStreamSynchronize(s));
  sg_status st = launch_upload(v, channel, timepoint, level, n,
                               reinterpret_cast<const int32_t*>(tmp + coff), dsrc, s);
  SG_HIP(hipFreeAsync(tmp, s));
  if (st != SG_OK) return st;
  v->pending[(size_t)timepoint * v->d.channels + channel] = 1;
  return SG_OK;
}

sg_status sg_build_lod(sg_volume* vol, int32_t channel, int32_t timepoint, void* hip_stream) {
  if (!vol) return fail(SG_ERR_INVALID_ARG, "sg_build_lod: NULL volume");
  Volume* v = &vol->v;
  if (v->cache)
    return fail(SG_ERR_UNSUPPORTED, "sg_build_lod: a cache volume holds no full level 0");
  if (channel < 0 || channel >= v->d.channels || timepoint < 0 || timepoint >= v->d.timepoints)
    return fail(SG_ERR_INVALID_ARG, "sg_build_lod: channel/timepoint out of range");
  DeviceGuard guard(v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  hipStream_t s = (hipStream_t)hip_stream;
  for (int L = 1; L < v->L; ++L) {
    sg_status st = launch_downsample(v, channel, timepoint, L, s);
    if (st != SG_OK) return st;
  }
  v->pending[(size_t)timepoint * v->d.channels + channel] = 1;
  return SG_OK;
}

sg_status sg_volume_commit(sg_volume* vol, void* hip_stream) {
  if (!vol) return fail(SG_ERR_INVALID_ARG, "sg_volume_commit: NULL volume");
  DeviceGuard guard(vol->v.d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  return commit(&vol->v, (hipStream_t)hip_stream);
}

sg_status sg_set_transfer_function(sg_volume* vol, int32_t channel, const float* rgba,
                                   int32_t n_entries, double domain_lo, double domain_hi) {
  if (!vol || !rgba) return fail(SG_ERR_INVALID_ARG, "sg_set_transfer_function: NULL argument");
  Volume* v = &vol->v;
  if (channel < 0 || channel >= v->d.channels)
    return fail(SG_ERR_INVALID_ARG, "sg_set_transfer_function: channel out of range");
  if (n_entries < 2 || n_entries > kMaxTfEntries)
    return fail(SG_ERR_INVALID_ARG, "sg_set_transfer_function: n_entries must be in [2, 1024]");
  if (!(std::isfinite(domain_lo) && std::isfinite(domain_hi) && domain_hi > domain_lo))
    return fail(SG_ERR_INVALID_ARG, "sg_set_transfer_function: need finite domain_lo < domain_hi");
  bool other = false;
  for (int c = 0; c < v->d.channels; ++c) other = other || (v->tf_set[c] && c != channel);
  if (other && n_entries != v->tf_n)
    return fail(SG_ERR_INVALID_ARG,
                "sg_set_transfer_function: every channel must use the same n_entries");
  for (int32_t i = 0; i < 4 * n_entries; ++i)
    if (!std::isfinite(rgba[i]) || ((i & 3) == 3 && rgba[i] < 0.0f))
      return fail(SG_ERR_INVALID_ARG,
                  "sg_set_transfer_function: entries must be finite, extinction >= 0");
  v->tf_n = n_entries;
  v->tf_host[channel].assign(rgba, rgba + 4 * n_entries);
  v->tf_lo[channel] = domain_lo;
  v->tf_hi[channel] = domain_hi;
  v->tf_set[channel] = true;
  v->tf_dirty = true;
  return SG_OK;
}

sg_status sg_set_kernel_timing(sg_volume* vol, int32_t enable) {
  if (!vol) return fail(SG_ERR_INVALID_ARG, "sg_set_kernel_timing: NULL volume");
  Volume* v = &vol->v;
  v->timing = enable != 0;
  for (hipEvent_t e : v->ev_rec) v->ev_free.push_back(e);
  v->ev_rec.clear();
  return SG_OK;
}

sg_status sg_get_kernel_timing(sg_volume* vol, int32_t* renders, double* cutmap_ms,
                               double* raycast_ms) {
  if (!vol || !renders || !cutmap_ms || !raycast_ms)
    return fail(SG_ERR_INVALID_ARG, "sg_get_kernel_timing: NULL argument");
  Volume* v = &vol->v;
  DeviceGuard guard(v->d.device);
  if (!guard.ok) return fail(SG_ERR_DEVICE, "cannot select device");
  double cut = 0.0, ray = 0.0;
  const size_t n = v->ev_rec.size() / 3;
  for (size_t i = 0; i < n; ++i) {
    float a = 0.f, b = 0.f;
    SG_HIP(hipEventSynchronize(v->ev_rec[3 * i + 2]));
    SG_HIP(hipEventElapsedTime(&a, v->ev_rec[3 * i], v->ev_rec[3 * i + 1]));
    SG_HIP(hipEventElapsedTime(&b, v->ev_rec[3 * i + 1], v->ev_rec[3 * i + 2]));
    cut += a;
    ray += b;
  }
  *renders = (int32_t)n;
  *cutmap_ms = cut;
  *raycast_ms = ray;
  for (hipEvent_t e : v->ev_rec) v->ev_free.push_back(e);
  v->ev_rec.clear();
  return SG_OK;
}

sg_status sg_volume_memory(const sg_volume* vol, uint64_t* bytes) {
  if (!vol || !bytes) return fail(SG_ERR_INVALID_ARG, "sg_volume_memory: NULL argument");
  *bytes = vol->v.bytes + (uint64_t)vol->v.cutmap_cap * 4 + (uint64_t)vol->v.view_cap +
           (uint64_t)vol->v.mb_words * 4;
  return SG_OK;
}

const char* sg_status_string(sg_status s) {
  switch (s) {
    case SG_OK: return "SG_OK";
    case SG_ERR_INVALID_ARG: return "SG_ERR_INVALID_ARG";
    case SG_ERR_OUT_OF_MEMORY: return "SG_ERR_OUT_OF_MEMORY";
    case SG_ERR_DEVICE: return "SG_ERR_DEVICE";
    case SG_ERR_STATE: return "SG_ERR_STATE";
    case SG_ERR_UNSUPPORTED: return "SG_ERR_UNSUPPORTED";
  }
  return "SG_ERR_UNKNOWN";
}

const char* sg_last_error(void) { return g_last_error.c_str(); }

int32_t sg_abi_version(void) { return SG_ABI_VERSION; }

}  // extern "C"
