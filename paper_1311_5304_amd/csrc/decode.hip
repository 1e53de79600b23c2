// Single-image kernel of the fused JPEG back half and its launcher.
//
// The image band (MCU rows [row0, row1)) is cut into strips of SX MCU
// columns and every strip into segments of consecutive sub-tile rows; each
// workgroup walks its segments with the pipelined SegmentDecoder.  The grid
// holds as many workgroups as the device keeps resident, so a workgroup that
// finishes early takes further segments rather than leaving its slot idle.
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
__global__ __launch_bounds__(C::NT, C::WAVES_PER_SIMD) void decode_segments(const ImageView im, const SegGrid sg) {
  __shared__ __align__(16) uint8_t lds[C::LDS_BYTES];
  // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a
  // contiguous run of segments (row-major over strips) so neighbouring
  // strips, whose chroma blocks each other's filter reads, share an L2.
  const int per_xcd = static_cast<int>(gridDim.x >> 3);
  const int v = static_cast<int>(blockIdx.x & 7u) * per_xcd + static_cast<int>(blockIdx.x >> 3);
  SegmentDecoder<C> dec(lds, im, static_cast<int>(threadIdx.x));
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

// Sub-tile shapes: a sub-tile's blocks fill whole waves (one block per lane)
// and the neighbour-column tasks of the fancy filter take the remaining
// lanes of the workgroup.
using Cfg420F = SegCfg<2, 2, true, 16, 2, 256>;
using Cfg420S = SegCfg<2, 2, false, 16, 2, 192>;
using Cfg422F = SegCfg<2, 1, true, 16, 2, 192>;
using Cfg422S = SegCfg<2, 1, false, 16, 2, 128>;
using Cfg444 = SegCfg<1, 1, false, 16, 4, 192>;

template <class C>
static hipError_t launch_cfg(const ImageView& im, int row0, int row1, int cu_count, const mjd_tuning& tu,
                             hipStream_t stream) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, decode_segments<C>, C::NT, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
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
  int grid = sg.segments < slots ? sg.segments : slots;
  if (tu.max_workgroups > 0 && grid > static_cast<int>(tu.max_workgroups)) grid = static_cast<int>(tu.max_workgroups);
  grid = (grid + 7) & ~7;
  hipLaunchKernelGGL(decode_segments<C>, dim3(grid), dim3(C::NT), 0, stream, im, sg);
  return hipGetLastError();
}

hipError_t launch_image(const ImageView& im, int row0, int row1, int hf, int vf, bool fancy, int cu_count,
                        const mjd_tuning& tu, hipStream_t stream) {
  if (hf == 1 && vf == 1) return launch_cfg<Cfg444>(im, row0, row1, cu_count, tu, stream);
  if (hf == 2 && vf == 1)
    return fancy ? launch_cfg<Cfg422F>(im, row0, row1, cu_count, tu, stream)
                 : launch_cfg<Cfg422S>(im, row0, row1, cu_count, tu, stream);
  return fancy ? launch_cfg<Cfg420F>(im, row0, row1, cu_count, tu, stream)
               : launch_cfg<Cfg420S>(im, row0, row1, cu_count, tu, stream);
}

}  // namespace mjd
