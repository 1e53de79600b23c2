// Single-image kernel of the fused JPEG back half and its launcher.
//
// The image band (MCU rows [row0, row1)) is cut into strips of SX MCU
// columns and every strip into segments of consecutive sub-tile rows; each
// workgroup walks its segments with the pipelined SegmentDecoder.  The grid
// holds as many workgroups as the device keeps resident, so a workgroup that
// finishes early takes further segments rather than leaving its slot idle.
#include <atomic>

#include "mjd_internal.h"
#include "segment.h"

namespace mjd {

struct SegGrid {
  int strips;     // strips of SX MCU columns
  int seg_rows;   // MCU rows per segment (a multiple of SY)
  int segs_per_strip;
  int segments;
  int row0, row1;
};

template <class C>
__device__ __forceinline__ void walk_segments(uint8_t* lds, const ImageView& im, const SegGrid& sg,
                                              const AanConsts* ak) {
  // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a
  // contiguous run of segments (row-major over strips) so neighbouring
  // strips, whose chroma blocks each other's filter reads, share an L2.
  const int per_xcd = static_cast<int>(gridDim.x >> 3);
  const int v = static_cast<int>(blockIdx.x & 7u) * per_xcd + static_cast<int>(blockIdx.x >> 3);
  SegmentDecoder<C> dec(lds, im, static_cast<int>(threadIdx.x), ak);
  for (int s = v; s < sg.segments; s += static_cast<int>(gridDim.x)) {
    const int sr = s / sg.strips;
    const int st = s - sr * sg.strips;
    SegmentRange r;
    r.mx0 = st * C::SX;
    r.r0 = sg.row0 + sr * sg.seg_rows;
    r.r1 = min(r.r0 + sg.seg_rows, sg.row1);
    dec.run(r);
  }
}

template <class C>
__global__ __launch_bounds__(C::NT, C::WAVES_PER_SIMD) void decode_segments(const ImageView im, const SegGrid sg) {
  __shared__ __align__(16) uint8_t lds[C::LDS_BYTES];
  walk_segments<C>(lds, im, sg, nullptr);
}

// The same walk with an AAN method's IDCT (its constants by value).
template <class C>
__global__ __launch_bounds__(C::NT, C::WAVES_PER_SIMD) void decode_segments_aan(const ImageView im, const SegGrid sg,
                                                                                const AanConsts ak) {
  __shared__ __align__(16) uint8_t lds[C::LDS_BYTES];
  walk_segments<C>(lds, im, sg, &ak);
}

// Workgroups of the kernel that stay resident on one CU, from the occupancy
// API once per device (every launch asks; the query costs microseconds).
constexpr int kMaxDevices = 64;
template <class C>
static hipError_t resident_per_cu(int* per_cu) {
  static std::atomic<int> cached[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < kMaxDevices) {
    const int c = cached[dev].load(std::memory_order_relaxed);
    if (c > 0) {
      *per_cu = c;
      return hipSuccess;
    }
  }
  *per_cu = 0;
  hipError_t e;
  if constexpr (C::ISLOW) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, decode_segments<C>, C::NT, 0);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, decode_segments_aan<C>, C::NT, 0);
  if (e == hipSuccess && *per_cu < 1) *per_cu = 1;
  if (e == hipSuccess && dev >= 0 && dev < kMaxDevices) cached[dev].store(*per_cu, std::memory_order_relaxed);
  return e;
}

template <class C>
static hipError_t launch_cfg(const ImageView& im, int row0, int row1, int cu_count, const mjd_tuning& tu,
                             hipStream_t stream) {
  int per_cu = 0;
  hipError_t e = resident_per_cu<C>(&per_cu);
  if (e != hipSuccess) return e;
  const int slots = per_cu * (cu_count > 0 ? cu_count : 256);
  SegGrid sg;
  sg.row0 = row0;
  sg.row1 = row1;
  sg.strips = (im.mcus_x + C::SX - 1) / C::SX;
  const int rows = row1 - row0;
  const int sub_rows = (rows + C::SY - 1) / C::SY;
  int seg_sub;
  if (tu.seg_subtiles > 0) {
    seg_sub = static_cast<int>(tu.seg_subtiles);
  } else {
    int want = (slots + sg.strips - 1) / sg.strips;  // segments per strip to fill the device once
    if (want < 1) want = 1;
    if (want > sub_rows) want = sub_rows;
    seg_sub = (sub_rows + want - 1) / want;
  }
  if (seg_sub > sub_rows) seg_sub = sub_rows;
  sg.seg_rows = seg_sub * C::SY;
  sg.segs_per_strip = (rows + sg.seg_rows - 1) / sg.seg_rows;
  sg.segments = sg.strips * sg.segs_per_strip;
  // the grid: every resident slot by default; a tuned count may be smaller
  // or larger (workgroups beyond the resident ones start as others finish)
  int grid = tu.workgroups > 0 ? static_cast<int>(tu.workgroups) : slots;
  if (grid > sg.segments) grid = sg.segments;
  grid = (grid + 7) & ~7;
  if constexpr (C::ISLOW) hipLaunchKernelGGL(decode_segments<C>, dim3(grid), dim3(C::NT), 0, stream, im, sg);
  else hipLaunchKernelGGL(decode_segments_aan<C>, dim3(grid), dim3(C::NT), 0, stream, im, sg, aan_consts());
  return hipGetLastError();
}

// Sub-tile shapes of each sampling class, the default first.  A sub-tile's
// blocks fill whole waves (one block per lane: SX * SY * blocks-per-MCU is a
// multiple of 64) and the neighbour-column tasks of the fancy filter take
// the remaining lanes of the workgroup; the 4:2:0 fancy class further needs
// its row pairs to fill the workgroup (NT = 4 * SY * 2 * SX), which leaves
// no shape with SX = 8.
struct Shape {
  int sx, sy, nt, lds_bytes;
  hipError_t (*launch)(const ImageView&, int, int, int, const mjd_tuning&, hipStream_t);
  hipError_t (*per_cu)(int*);
};

template <class C>
constexpr Shape shape_of() {
  return Shape{C::SX, C::SY, C::NT, C::LDS_BYTES, &launch_cfg<C>, &resident_per_cu<C>};
}

static constexpr Shape k420F[] = {shape_of<SegCfg<2, 2, true, 16, 2, 256>>(), shape_of<SegCfg<2, 2, true, 32, 1, 256>>(),
                                  shape_of<SegCfg<2, 2, true, 16, 4, 512>>()};
static constexpr Shape k420S[] = {shape_of<SegCfg<2, 2, false, 16, 2, 192>>(), shape_of<SegCfg<2, 2, false, 32, 1, 192>>(),
                                  shape_of<SegCfg<2, 2, false, 8, 4, 192>>(), shape_of<SegCfg<2, 2, false, 16, 4, 384>>()};
static constexpr Shape k422F[] = {shape_of<SegCfg<2, 1, true, 16, 2, 192>>(), shape_of<SegCfg<2, 1, true, 32, 1, 192>>(),
                                  shape_of<SegCfg<2, 1, true, 8, 4, 256>>(), shape_of<SegCfg<2, 1, true, 16, 1, 128>>()};
static constexpr Shape k422S[] = {shape_of<SegCfg<2, 1, false, 16, 2, 128>>(), shape_of<SegCfg<2, 1, false, 32, 1, 128>>(),
                                  shape_of<SegCfg<2, 1, false, 8, 4, 128>>(), shape_of<SegCfg<2, 1, false, 16, 4, 256>>()};
static constexpr Shape k444[] = {shape_of<SegCfg<1, 1, false, 16, 4, 192>>(), shape_of<SegCfg<1, 1, false, 32, 2, 192>>(),
                                 shape_of<SegCfg<1, 1, false, 8, 8, 192>>(), shape_of<SegCfg<1, 1, false, 16, 8, 384>>()};

template <size_t N>
static void pick(const Shape (&l)[N], const Shape** list, int* n) {
  *list = l;
  *n = static_cast<int>(N);
}

// The shape list of a sampling class (hf, vf in {1, 2}).
static void class_shapes(int hf, int vf, bool fancy, const Shape** list, int* n) {
  if (hf == 1 && vf == 1) return pick(k444, list, n);
  if (hf == 2 && vf == 1) return fancy ? pick(k422F, list, n) : pick(k422S, list, n);
  return fancy ? pick(k420F, list, n) : pick(k420S, list, n);
}

int shape_count(int hf, int vf, bool fancy) {
  const Shape* l;
  int n;
  class_shapes(hf, vf, fancy, &l, &n);
  return n;
}

hipError_t shape_info(int hf, int vf, bool fancy, int index, int* sx, int* sy, int* nt, int* lds_bytes, int* per_cu) {
  const Shape* l;
  int n;
  class_shapes(hf, vf, fancy, &l, &n);
  const Shape& s = l[index];
  *sx = s.sx;
  *sy = s.sy;
  *nt = s.nt;
  *lds_bytes = s.lds_bytes;
  return s.per_cu(per_cu);
}

// The decoder variants on the fused path: every sampling (luma (1,1), (2,1),
// (1,2), (2,2), (4,1)) with every IDCT method, one sub-tile shape each
// (islow's 4:4:4 / 4:2:2 / 4:2:0 are the single-image kernel's shape lists).
// A factor of 4 is replicated in both modes.
template <int M>
static hipError_t launch_variant_method(const ImageView& im, int hf, int vf, bool fancy, int cu_count,
                                       const mjd_tuning& tu, hipStream_t stream) {
  const int rows = im.mcus_y;
  if (hf == 4) return launch_cfg<SegCfg<4, 1, false, 8, 4, 192, M>>(im, 0, rows, cu_count, tu, stream);
  if (hf == 1 && vf == 2)
    return fancy ? launch_cfg<SegCfg<1, 2, true, 16, 2, 128, M>>(im, 0, rows, cu_count, tu, stream)
                 : launch_cfg<SegCfg<1, 2, false, 16, 2, 128, M>>(im, 0, rows, cu_count, tu, stream);
  if constexpr (M == 0) {
    return launch_image(im, 0, rows, hf, vf, fancy, cu_count, tu, stream);
  } else {
    if (hf == 1) return launch_cfg<SegCfg<1, 1, false, 16, 4, 192, M>>(im, 0, rows, cu_count, tu, stream);
    if (vf == 1)
      return fancy ? launch_cfg<SegCfg<2, 1, true, 16, 2, 192, M>>(im, 0, rows, cu_count, tu, stream)
                   : launch_cfg<SegCfg<2, 1, false, 16, 2, 128, M>>(im, 0, rows, cu_count, tu, stream);
    return fancy ? launch_cfg<SegCfg<2, 2, true, 16, 2, 256, M>>(im, 0, rows, cu_count, tu, stream)
                 : launch_cfg<SegCfg<2, 2, false, 16, 2, 192, M>>(im, 0, rows, cu_count, tu, stream);
  }
}

hipError_t launch_image(const ImageView& im, int row0, int row1, int hf, int vf, bool fancy, int cu_count,
                        const mjd_tuning& tu, hipStream_t stream) {
  const Shape* l;
  int n;
  class_shapes(hf, vf, fancy, &l, &n);
  const int i = static_cast<int>(tu.shape) < n ? static_cast<int>(tu.shape) : 0;
  return l[i].launch(im, row0, row1, cu_count, tu, stream);
}

hipError_t launch_variant(const ImageView& im, int hf, int vf, bool fancy, int idct, int cu_count,
                          const mjd_tuning& tu, hipStream_t stream) {
  switch (idct) {
    case 0: return launch_variant_method<0>(im, hf, vf, fancy, cu_count, tu, stream);
    case 1: return launch_variant_method<1>(im, hf, vf, fancy, cu_count, tu, stream);
    default: return launch_variant_method<2>(im, hf, vf, fancy, cu_count, tu, stream);
  }
}

}  // namespace mjd
