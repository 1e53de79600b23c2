// GPU entropy decoding of many baseline scans: one lane per restart interval.
//
// The host plans the work:
// - it checks every job;
// - it builds each job's Huffman tables in the layout the kernel copies to
//   LDS;
// - it lists the restart intervals, sorts each job's list by length, and
//   cuts it into items of at most 256 intervals, so an item never spans two
//   jobs; items go longest first.
// A persistent kernel pops items from a device counter. A workgroup loads
// the tables of the item's job into LDS (only when the job changes). Each
// lane then decodes one interval with the bit reader and block decoder of
// entropy_lane.h. Blocks are scattered into a per-lane LDS buffer and stored
// whole (128 B) in MCU order, the layout mjd_decode reads. Each interval's
// status goes to a device array; the last workgroup out rearms the counter.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "entropy_lane.h"
#include "host_jpeg.h"
#include "mjd_internal.h"

namespace mjd {
namespace gent {

struct GJob {
  const uint8_t* jpg;
  int16_t* coef;
  const GTables* tables;
  uint32_t lim;        // stream bytes, rounded up to 16 (chunk loads stay below)
  int32_t bpm;         // blocks per MCU
  uint32_t comp_bits;  // component of block b of an MCU in bits 2b..2b+1
  uint32_t tsel;       // table slots of each component (plan_gtables)
};

struct GItem {
  uint32_t job, first, count;
  uint32_t bytes;  // stream bytes of its longest interval
};

constexpr int kThreads = 256;
constexpr uint64_t kMaxStream = 0xFFFFFF00u;  // stream offsets are 32-bit

static int tables_for(const mjd_scan& scan, GTables* g, uint32_t* tsel) {
  switch (plan_gtables(scan, g, tsel)) {
    case kTableOk:
      return MJD_OK;
    case kTableUndefined:
      return fail(MJD_ECORRUPT, "scan uses an undefined Huffman table");
    case kTableTooMany:
      return fail(MJD_ECORRUPT, "Huffman table with more than 256 symbols");
    case kPlanTooManyTables:
      return fail(MJD_EUNSUPPORTED, "scan uses more than %d distinct Huffman tables (baseline uses at most 4); "
                                    "decode it on the host", kTableSlots);
    default:
      return fail(MJD_ECORRUPT, "Huffman code lengths overfill the code space");
  }
}

typedef __attribute__((address_space(3))) uint8_t lds8;
typedef __attribute__((address_space(3))) uint16_t lds16;
typedef __attribute__((address_space(3))) uint32_t lds32;
typedef __attribute__((address_space(1))) const uint8_t gin8;
typedef __attribute__((address_space(1))) const uint32_t gin32;
typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) v4i_t gout128;
typedef __attribute__((address_space(1))) const v4i_t gin128;
typedef __attribute__((address_space(3))) v4i_t lds128;

// Tables and the zig-zag map, in LDS.
struct DevTab {
  const __attribute__((address_space(3))) GHuff* tab;
  const lds8* natural;
  __device__ uint32_t fast(int t, int i) const { return tab[t].fast[i]; }
  __device__ int lim(int t, int l) const { return tab[t].lim[l]; }
  __device__ int valoff(int t, int l) const { return tab[t].valoff[l]; }
  __device__ int val(int t, int i) const { return tab[t].vals[i]; }
  __device__ int nat(int k) const { return natural[k]; }
};

// Per-lane LDS buffers (128-byte blocks, kRing-byte rings) sit one buffer
// apart, so their 16-byte chunks are rotated by the lane number: the lanes
// of a wave then spread a 16-byte access at the same offset over the banks.
template <uint32_t kBytes>
__device__ inline uint32_t swz(uint32_t off, uint32_t rot) {
  static_assert(kBytes >= 16 && (kBytes & (kBytes - 1)) == 0, "buffers of a power-of-two number of chunks");
  return (((off >> 4) + rot) & (kBytes / 16 - 1)) << 4 | (off & 15u);
}

// The block being decoded: 128 bytes of LDS per lane, stored whole (eight
// 16-byte stores) to the next block of the interval and cleared.  The
// stores are non-temporal: the coefficients are not read again by this
// kernel, and written lines that stayed in the L2 would evict the lines of
// the lanes' streams, which are then fetched again for every 16-byte chunk
// (about 5 times the entropy-coded bytes instead of about 1.3).
struct DevBlk {
  lds8* buf;
  gout128* dst;
  uint32_t rot;
  __device__ void put(int idx, int v) {
    *reinterpret_cast<lds16*>(buf + swz<128>(static_cast<uint32_t>(idx) * 2, rot)) = static_cast<uint16_t>(v);
  }
  __device__ void finish() {
#pragma unroll
    for (int i = 0; i < 8; ++i) __builtin_nontemporal_store(*reinterpret_cast<lds128*>(buf + swz<128>(16u * i, rot)), &dst[i]);
#pragma unroll
    for (int i = 0; i < 8; ++i) reinterpret_cast<lds128*>(buf)[i] = v4i_t{0, 0, 0, 0};
    dst += 8;
  }
};

// The lane's stream: 16-byte chunk loads from global memory, held in two
// register slots until the next refill writes them to the lane's 128-byte
// LDS ring, from which every stream byte is read.
struct DevMem {
  gin8* jpg;
  lds8* ring;
  uint32_t rot;
  v4i_t c0, c1;
  __device__ void g_chunk(uint32_t p, int slot) {
    const v4i_t v = *reinterpret_cast<gin128*>(jpg + p);
    if (slot) c1 = v;
    else c0 = v;
  }
  __device__ void commit(int slot, uint32_t off) { *reinterpret_cast<lds128*>(ring + swz<kRing>(off, rot)) = slot ? c1 : c0; }
  __device__ uint32_t r_dword(uint32_t off) const { return *reinterpret_cast<const lds32*>(ring + swz<kRing>(off, rot)); }
};

__global__ __launch_bounds__(kThreads) void entropy_kernel(const GJob* __restrict__ jobs,
                                                           const Interval* __restrict__ ivs,
                                                           const GItem* __restrict__ items, int n_items,
                                                           uint32_t* __restrict__ status, unsigned* counters) {
  __shared__ __align__(16) GTables tabs;
  __shared__ __align__(16) uint32_t blocks[kThreads * 32];
  __shared__ __align__(16) uint8_t rings[kThreads * kRing];
  __shared__ int s_next;
  const int tid = static_cast<int>(threadIdx.x);
  {
    lds128* b = reinterpret_cast<lds128*>((lds8*)blocks + tid * 128);
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = v4i_t{0, 0, 0, 0};
  }
  int cur_job = -1;
  for (;;) {
    if (tid == 0) s_next = static_cast<int>(atomicAdd(&counters[0], 1u));
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_next);
    __syncthreads();  // every lane has read s_next (and finished the last item)
    if (it >= n_items) break;
    const GItem item = items[it];
    const int job = __builtin_amdgcn_readfirstlane(static_cast<int>(item.job));
    if (job != cur_job) {
      gin128* src = (gin128*)jobs[job].tables;
      lds128* dst = (lds128*)&tabs;
      for (int i = tid; i < static_cast<int>(sizeof(GTables) / 16); i += kThreads) dst[i] = src[i];
      __syncthreads();
      cur_job = job;
    }
    if (tid < static_cast<int>(item.count)) {
      const GJob& jb = jobs[job];
      const Interval iv = ivs[item.first + static_cast<uint32_t>(tid)];
      DevTab tab{(const __attribute__((address_space(3))) GHuff*)tabs.t, (const lds8*)tabs.nat};
      const uint32_t rot = static_cast<uint32_t>(tid) & 7u;
      DevBlk blk{(lds8*)blocks + tid * 128, (gout128*)(jb.coef + iv.mcu0 * static_cast<uint64_t>(jb.bpm) * 64), rot};
      DevMem mem{(gin8*)jb.jpg, (lds8*)rings + tid * kRing, rot, v4i_t{0, 0, 0, 0}, v4i_t{0, 0, 0, 0}};
      const uint32_t st = decode_interval(tab, blk, mem, jb.lim, iv, jb.bpm, jb.comp_bits, jb.tsel);
      if (st != kOk) {  // leave the block buffer clear for the next interval
        lds128* b = reinterpret_cast<lds128*>(blk.buf);
#pragma unroll
        for (int i = 0; i < 8; ++i) b[i] = v4i_t{0, 0, 0, 0};
      }
      status[item.first + static_cast<uint32_t>(tid)] = st;
    }
  }
  // the last workgroup out rearms the queue for the next launch
  if (tid == 0) {
    __threadfence();
    const unsigned done = atomicAdd(&counters[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&counters[0], 0u);
      atomicExch(&counters[1], 0u);
    }
  }
}

}  // namespace gent
}  // namespace mjd

struct mjd_entropy_batch {
  mjd_ctx* ctx = nullptr;
  uint32_t n_jobs = 0;
  uint32_t n_intervals = 0;
  uint32_t n_items = 0;
  int grid = 0;
  mjd::gent::GJob* d_jobs = nullptr;
  mjd::gent::GTables* d_tables = nullptr;
  mjd::gent::Interval* d_ivs = nullptr;
  mjd::gent::GItem* d_items = nullptr;
  uint32_t* d_status = nullptr;
  unsigned* d_counters = nullptr;
  std::vector<uint32_t> first_interval;  // per job, into the interval list
  std::vector<uint32_t> iv_index;        // per listed interval, its number in its scan
  uint64_t pixels = 0, bytes = 0;
};

namespace mjd {
namespace gent {

static void free_batch(mjd_entropy_batch* b) {
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->d_tables) (void)hipFree(b->d_tables);
  if (b->d_ivs) (void)hipFree(b->d_ivs);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_status) (void)hipFree(b->d_status);
  if (b->d_counters) (void)hipFree(b->d_counters);
}

static int build(mjd_ctx* ctx, const mjd_entropy_job* jobs, size_t n, mjd_entropy_batch* b) {
  if (n == 0) return fail(MJD_EINVAL, "empty entropy batch");
  if (n > (1u << 24)) return fail(MJD_EINVAL, "entropy batch of %zu jobs too large", n);
  std::vector<GJob> gj(n);
  std::vector<GTables> gt(n);
  std::vector<Interval> ivs;
  std::vector<GItem> items;
  b->first_interval.resize(n);
  for (size_t j = 0; j < n; ++j) {
    const mjd_entropy_job& J = jobs[j];
    if (!J.scan || !J.h_offsets || !J.d_jpg || !J.d_coef)
      return fail(MJD_EINVAL, "job %zu: null scan, offsets, stream or coefficient pointer", j);
    if ((reinterpret_cast<uintptr_t>(J.d_jpg) & 15) || (reinterpret_cast<uintptr_t>(J.d_coef) & 15))
      return fail(MJD_EINVAL, "job %zu: stream or coefficients not 16-byte aligned", j);
    if (J.len > kMaxStream) return fail(MJD_EINVAL, "job %zu: stream of %llu bytes is too long", j,
                                        static_cast<unsigned long long>(J.len));
    host::ScanLayout L;
    int rc = host::scan_layout(J.scan, &L);
    if (rc != MJD_OK) {
      const std::string why = mjd_last_error();
      return fail(rc, "job %zu: %s", j, why.c_str());
    }
    if (L.bpm > 8) return fail(MJD_EINVAL, "job %zu: %d blocks per MCU", j, L.bpm);
    rc = tables_for(*J.scan, &gt[j], &gj[j].tsel);
    if (rc != MJD_OK) {
      const std::string why = mjd_last_error();
      return fail(rc, "job %zu: %s", j, why.c_str());
    }
    memcpy(gt[j].nat, host::zigzag_to_natural(), 64);
    gj[j].jpg = J.d_jpg;
    gj[j].coef = J.d_coef;
    gj[j].lim = static_cast<uint32_t>((J.len + 15) & ~uint64_t{15});
    gj[j].bpm = L.bpm;
    gj[j].comp_bits = 0;
    for (int i = 0; i < L.bpm; ++i) gj[j].comp_bits |= static_cast<uint32_t>(L.comp_of[i]) << (2 * i);
    // the intervals: byte ranges from the restart index, checked against the stream
    const uint32_t ni = J.scan->n_intervals;
    const uint64_t ri = J.scan->restart_interval ? J.scan->restart_interval : L.n_mcus;
    const uint64_t* off = J.h_offsets;
    if (off[ni] > J.len) return fail(MJD_EINVAL, "job %zu: restart index past the stream end", j);
    b->first_interval[j] = static_cast<uint32_t>(ivs.size());
    for (uint32_t s = 0; s < ni; ++s) {
      if (off[s + 1] < off[s] + 2) return fail(MJD_EINVAL, "job %zu: restart index not increasing", j);
      Interval iv;
      iv.start = static_cast<uint32_t>(off[s]);
      iv.end = static_cast<uint32_t>(off[s + 1] - 2);
      iv.index = s;
      iv.mcu0 = s * ri;
      iv.n_mcus = static_cast<uint32_t>(std::min<uint64_t>(ri, L.n_mcus - iv.mcu0));
      ivs.push_back(iv);
    }
    // A lane's decode time follows its interval's length, and a wave (and a
    // workgroup) lasts as long as its longest interval: sort the job's
    // intervals longest first so that each item holds intervals of similar
    // length.
    const auto first = ivs.begin() + b->first_interval[j];
    std::stable_sort(first, ivs.end(),
                     [](const Interval& x, const Interval& y) { return x.end - x.start > y.end - y.start; });
    for (uint32_t s = 0; s < ni; s += kThreads) {
      const Interval& lead = ivs[b->first_interval[j] + s];
      items.push_back(GItem{static_cast<uint32_t>(j), b->first_interval[j] + s, std::min<uint32_t>(kThreads, ni - s),
                            lead.end - lead.start});
    }
    b->pixels += static_cast<uint64_t>(J.scan->frame.width) * J.scan->frame.height;
    b->bytes += J.len;
    if (ivs.size() > 0x7FFFFFF0u) return fail(MJD_EINVAL, "entropy batch holds too many intervals");
  }
  // longest items first, so that the last ones to start are short
  std::stable_sort(items.begin(), items.end(), [](const GItem& x, const GItem& y) { return x.bytes > y.bytes; });
  b->iv_index.resize(ivs.size());
  for (size_t i = 0; i < ivs.size(); ++i) b->iv_index[i] = ivs[i].index;
  b->n_jobs = static_cast<uint32_t>(n);
  b->n_intervals = static_cast<uint32_t>(ivs.size());
  b->n_items = static_cast<uint32_t>(items.size());
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, entropy_kernel, kThreads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  b->grid = std::min<int>(static_cast<int>(items.size()), per_cu * (ctx->cu_count > 0 ? ctx->cu_count : 256));
  if (hipMalloc(&b->d_tables, n * sizeof(GTables)) != hipSuccess ||
      hipMalloc(&b->d_jobs, n * sizeof(GJob)) != hipSuccess ||
      hipMalloc(&b->d_ivs, ivs.size() * sizeof(Interval)) != hipSuccess ||
      hipMalloc(&b->d_items, items.size() * sizeof(GItem)) != hipSuccess ||
      hipMalloc(&b->d_status, ivs.size() * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc(&b->d_counters, 2 * sizeof(unsigned)) != hipSuccess)
    return fail(MJD_ENOMEM, "device allocation for the entropy batch tables failed");
  for (size_t j = 0; j < n; ++j) gj[j].tables = b->d_tables + j;
  if (hipMemcpy(b->d_tables, gt.data(), n * sizeof(GTables), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_jobs, gj.data(), n * sizeof(GJob), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_ivs, ivs.data(), ivs.size() * sizeof(Interval), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->d_items, items.data(), items.size() * sizeof(GItem), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(b->d_status, 0, ivs.size() * sizeof(uint32_t)) != hipSuccess ||
      hipMemset(b->d_counters, 0, 2 * sizeof(unsigned)) != hipSuccess)
    return fail(MJD_EDEVICE, "uploading the entropy batch tables failed");
  return MJD_OK;
}

}  // namespace gent
}  // namespace mjd

extern "C" {

int mjd_entropy_batch_create(mjd_ctx* ctx, const mjd_entropy_job* jobs, size_t n, mjd_entropy_batch** out) {
  if (!ctx || !out) return mjd::fail(MJD_EINVAL, "null context or out-pointer");
  *out = nullptr;
  if (!jobs && n) return mjd::fail(MJD_EINVAL, "null jobs");
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
    return mjd::fail(MJD_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
  mjd_entropy_batch* b = new (std::nothrow) mjd_entropy_batch;
  if (!b) return mjd::fail(MJD_ENOMEM, "entropy batch allocation failed");
  b->ctx = ctx;
  int rc = mjd::gent::build(ctx, jobs, n, b);
  if (cur != ctx->device) (void)hipSetDevice(cur);
  if (rc != MJD_OK) {
    mjd::gent::free_batch(b);
    delete b;
    return rc;
  }
  *out = b;
  return MJD_OK;
}

int mjd_entropy_batch_launch(mjd_entropy_batch* b, void* stream) {
  if (!b) return mjd::fail(MJD_EINVAL, "null entropy batch");
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != b->ctx->device && hipSetDevice(b->ctx->device) != hipSuccess)
    return mjd::fail(MJD_EDEVICE, "hipSetDevice(%d) failed", b->ctx->device);
  hipLaunchKernelGGL(mjd::gent::entropy_kernel, dim3(b->grid), dim3(mjd::gent::kThreads), 0,
                     static_cast<hipStream_t>(stream), b->d_jobs, b->d_ivs, b->d_items, static_cast<int>(b->n_items),
                     b->d_status, b->d_counters);
  hipError_t e = hipGetLastError();
  if (cur != b->ctx->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return mjd::fail(MJD_EDEVICE, "entropy kernel launch failed: %s", hipGetErrorString(e));
  return MJD_OK;
}

int mjd_entropy_batch_status(mjd_entropy_batch* b, int64_t* bad_job) {
  if (!b) return mjd::fail(MJD_EINVAL, "null entropy batch");
  if (bad_job) *bad_job = -1;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != b->ctx->device && hipSetDevice(b->ctx->device) != hipSuccess)
    return mjd::fail(MJD_EDEVICE, "hipSetDevice(%d) failed", b->ctx->device);
  std::vector<uint32_t> st(b->n_intervals);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(st.data(), b->d_status, st.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
  if (cur != b->ctx->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return mjd::fail(MJD_EDEVICE, "reading the entropy status failed: %s", hipGetErrorString(e));
  for (uint32_t i = 0; i < b->n_intervals; ++i) {
    if (!st[i]) continue;
    const auto it = std::upper_bound(b->first_interval.begin(), b->first_interval.end(), i);
    const int64_t job = static_cast<int64_t>(it - b->first_interval.begin()) - 1;
    if (bad_job) *bad_job = job;
    static const char* what[] = {"", "an invalid Huffman code", "a coefficient run past the end of a block",
                                 "an interval that ends before its last MCU"};
    return mjd::fail(MJD_ECORRUPT, "job %lld, restart interval %u: %s", static_cast<long long>(job),
                     b->iv_index[i], what[st[i] < 4 ? st[i] : 1]);
  }
  return MJD_OK;
}

int mjd_entropy_batch_info(const mjd_entropy_batch* b, uint32_t* intervals, uint32_t* workgroups, uint64_t* bytes) {
  if (!b) return mjd::fail(MJD_EINVAL, "null entropy batch");
  if (intervals) *intervals = b->n_intervals;
  if (workgroups) *workgroups = static_cast<uint32_t>(b->grid);
  if (bytes) *bytes = b->bytes;
  return MJD_OK;
}

void mjd_entropy_batch_destroy(mjd_entropy_batch* b) {
  if (!b) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != b->ctx->device) (void)hipSetDevice(b->ctx->device);
  (void)hipDeviceSynchronize();
  mjd::gent::free_batch(b);
  if (cur != b->ctx->device) (void)hipSetDevice(cur);
  delete b;
}

}  // extern "C"
