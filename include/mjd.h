/*
 * mjd.h - C ABI of the MI355X (gfx950) JPEG back-half decoder.
 *
 * The library runs the data-parallel part of baseline JPEG decoding that
 * Sodsong et al. (PMAM'14) move off the CPU: dequantisation, the 8x8
 * inverse DCT, chroma upsampling and YCbCr->RGB colour conversion (paper
 * Sec. 2, Fig. 1; Sec. 4).  As in the paper's statement of the problem
 * (Sec. 7, Sec. 4), the input is an array of 16-bit quantised DCT
 * coefficients, the image's quantisation tables (Sec. 2) and the
 * components' sampling factors (Sec. 2); the output is interleaved 8-bit
 * RGB, one byte per channel, rows top to bottom (Sec. 4.3, Fig. 4b, Fig. 5).
 * All stages run as one fused HIP kernel; no intermediate plane is written
 * to device memory.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Status: every function returns MJD_OK (0) or a negative mjd_status.
 *   mjd_last_error() returns a thread-local message for the last failure.
 *   No C++ exception crosses this interface.
 * - Pointers named d_* are device pointers (HIP global memory on the
 *   context's device); h_* are host pointers.  The caller owns every buffer;
 *   the library keeps no pointer after the enqueued work completes.
 * - Device calls are asynchronous on the caller's HIP stream (passed as
 *   void*; NULL means the default stream).  Argument validation happens
 *   synchronously before anything is enqueued; on an error nothing is
 *   enqueued.
 * - Coefficient layout (MCU order): MCUs in raster order; inside an MCU
 *   the luma blocks (v rows x h columns, raster), then one Cb block, then
 *   one Cr block.  Each block is 64 int16 in natural order, index
 *   8*row + col, row = vertical frequency (already de-zig-zagged).  The
 *   padding MCUs at the right and bottom edges are present and complete.
 *   The coefficient array must be 16-byte aligned.
 * - Quantisation tables: uint16[4][64] in natural order; component c uses
 *   table qsel[c].  Entries 1..255 for baseline data.
 * - Numeric domain: with |coefficient * Q| <= 1155 for every coefficient
 *   (every block produced from 8-bit samples has |F| <= 1024, so
 *   |c * Q| <= 1024 + Q/2 <= 1151), every intermediate of the fixed-point
 *   IDCT fits in int32 and the result is the defined one.  Outside that
 *   domain the call is still memory-safe but its output is unspecified.
 * - Output: RGB8 rows of `pitch` bytes (pitch >= 3 * width); only the
 *   bytes of the decoded rows' first 3 * width columns are written.
 */
#ifndef MJD_H
#define MJD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mjd_status {
  MJD_OK = 0,
  MJD_EINVAL = -1,       /* bad argument (null pointer, size, alignment, range) */
  MJD_EUNSUPPORTED = -2, /* valid JPEG parameters this library does not decode */
  MJD_ENOMEM = -3,       /* a host or device allocation failed */
  MJD_EDEVICE = -4,      /* a HIP runtime call failed */
  MJD_ECORRUPT = -5,     /* malformed bitstream */
  MJD_EBUDGET = -6       /* request larger than the configured memory budget */
} mjd_status;

typedef enum mjd_upsample {
  /* Replicate each chroma sample over its 2x1 or 2x2 group. */
  MJD_UPSAMPLE_SIMPLE = 0,
  /* Triangle ("fancy") filter: paper Sec. 4.2, Algorithm 1 over whole
   * component rows for 4:2:2; for 4:2:0 an unrounded vertical 3:1 sum
   * followed by the horizontal 3:1 filter, (3S[k] + S[k-1] + 8) >> 4 on even
   * and (3S[k] + S[k+1] + 7) >> 4 on odd outputs.  Neighbours are clamped
   * at the true component edge ceil(W*h/hmax) x ceil(H*v/vmax). */
  MJD_UPSAMPLE_FANCY = 1
} mjd_upsample;

/* Frame description (paper Sec. 2: dimensions and component subsampling
 * come from the frame header).  Components: 0 = Y, 1 = Cb, 2 = Cr.
 * Supported: (h[0], v[0]) in {(1,1), (2,1), (2,2)} (4:4:4, 4:2:2, 4:2:0),
 * h[1] = v[1] = h[2] = v[2] = 1; width and height 1..65535; qsel 0..3. */
typedef struct mjd_frame {
  uint32_t width;
  uint32_t height;
  uint8_t h[3];
  uint8_t v[3];
  uint8_t qsel[3];
  uint8_t reserved; /* must be 0 */
} mjd_frame;

/* MCU geometry (paper Sec. 2: an MCU is 8x8 pixels for 4:4:4 and 16x8 for
 * 4:2:2; 16x16 for 4:2:0).  comp_w/comp_h are the true component sizes
 * ceil(W*h_c/hmax) x ceil(H*v_c/vmax). */
typedef struct mjd_geometry {
  uint32_t mcu_w, mcu_h;
  uint32_t mcus_x, mcus_y;
  uint32_t blocks_per_mcu;
  uint32_t comp_w[3];
  uint32_t comp_h[3];
  uint64_t n_blocks;
} mjd_geometry;

/* Opaque per-device context: owns the library's device workspace
 * (batch descriptor tables, work-queue counters), its HIP graphs and its
 * tuned launch choices.  Calls on distinct contexts are thread-safe; one
 * context must not be used from two threads at once. */
typedef struct mjd_ctx mjd_ctx;

/* Launch shape of the decode kernels (paper Sec. 4.1 and Sec. 5: the best
 * work-group size is hardware specific and chosen by profiling).  The image
 * is cut into strips of sub-tiles; a workgroup walks a segment of
 * `seg_subtiles` consecutive sub-tile rows of one strip, prefetching the
 * next sub-tile while it decodes the current one, and takes further
 * segments when it finishes one.
 *   seg_subtiles  sub-tile rows per segment; 0: the automatic choice
 *                 (single image: enough segments to fill every resident
 *                 slot once; batch: about four segments per slot).
 *   workgroups    workgroups launched; 0: as many as the device keeps
 *                 resident.  A larger count is allowed: the extra
 *                 workgroups start as resident ones finish.  Never more
 *                 than there are segments.
 *   shape         sub-tile shape of the single-image kernel, an index into
 *                 the sampling class's list (mjd_shape_count /
 *                 mjd_shape_info); 0 is the class's default, and an index
 *                 past the end of a class's list selects that default.  The
 *                 batch kernel has one fixed shape per class.
 * The values change only speed, never the output. */
typedef struct mjd_tuning {
  uint32_t seg_subtiles;
  uint32_t workgroups;
  uint32_t shape;
} mjd_tuning;

/* One sub-tile shape of the single-image kernel. */
typedef struct mjd_shape {
  uint32_t mcus_x;          /* sub-tile width in MCUs */
  uint32_t mcus_y;          /* sub-tile height in MCUs */
  uint32_t threads;         /* lanes per workgroup */
  uint32_t lds_bytes;       /* LDS per workgroup */
  uint32_t resident_per_cu; /* workgroups one compute unit holds at once */
  uint32_t cu_count;        /* compute units of the context's device */
} mjd_shape;

/* Create a context on HIP device `device` (makes it current while creating). */
int mjd_ctx_create(mjd_ctx** out, int device);
/* Release a context and its device workspace.  Synchronises the device. */
void mjd_ctx_destroy(mjd_ctx* ctx);

/* Set / read the context's launch shape (see mjd_tuning).  Host only.
 * Returns MJD_EINVAL for null pointers, seg_subtiles > 65536,
 * workgroups > 2^20 or shape > 255. */
int mjd_ctx_set_tuning(mjd_ctx* ctx, const mjd_tuning* tuning);
int mjd_ctx_get_tuning(const mjd_ctx* ctx, mjd_tuning* tuning);

/* The sub-tile shapes the autotuner searches (paper Sec. 4.1: work-group
 * size per platform by profiling) for the sampling class of luma factors
 * h x v (1x1, 2x1 or 2x2, chroma 1x1) and upsampling mode.
 * mjd_shape_count: host only, writes the number of shapes to *count.
 * mjd_shape_info: fills *out for shape `index`, with the occupancy on the
 * context's device.  Return MJD_EINVAL for null pointers, an unknown mode or
 * an index past the list, MJD_EUNSUPPORTED for other sampling factors. */
int mjd_shape_count(uint32_t h, uint32_t v, int upsample, uint32_t* count);
int mjd_shape_info(mjd_ctx* ctx, uint32_t h, uint32_t v, int upsample, uint32_t index, mjd_shape* out);

/* Host-only: validate `frame` and compute its geometry.  Needs no GPU.
 * Returns MJD_EINVAL for null pointers or out-of-range fields and
 * MJD_EUNSUPPORTED for valid-but-unsupported sampling factors. */
int mjd_geometry_of(const mjd_frame* frame, mjd_geometry* out);

/* Decode MCU rows [mcu_row0, mcu_row1) of one image (paper Sec. 4: dequantise
 * + IDCT (Sec. 4.1, Eqs. 1-2), upsampling (Sec. 4.2), colour conversion
 * (Sec. 4.3), fused into one launch; the paper's horizontal chunks (Sec. 4.5)
 * are MCU-row bands here).
 *   d_coef: n_blocks * 64 int16 in MCU order (see above), 16-byte aligned.
 *   d_qt:   uint16[4][64] natural order, 2-byte aligned.
 *   d_rgb:  image base (row 0); rows [mcu_h*row0, min(H, mcu_h*row1)) are
 *           written, each 3*width bytes at d_rgb + y*pitch.
 * Reads blocks of MCU rows [row0, row1) only, plus, for fancy 4:2:0, the
 * chroma blocks of MCU rows row0-1 and row1 when they exist, and for fancy
 * 4:2:0 / 4:2:2 the chroma blocks of the horizontally adjacent MCUs; those
 * must already hold valid data.  Requires 0 <= row0 < row1 <= mcus_y. */
int mjd_decode(mjd_ctx* ctx, const mjd_frame* frame, const int16_t* d_coef,
               const uint16_t* d_qt, int upsample, uint8_t* d_rgb, size_t pitch,
               uint32_t mcu_row0, uint32_t mcu_row1, void* stream);

/* The same decode on host cores: the CPU side of the paper's CPU-GPU
 * partitioning (Sec. 5.2), which gives the CPU the image rows the GPU does
 * not take.  Same arithmetic and bytes as mjd_decode; host pointers; rows
 * [mcu_h*row0, min(H, mcu_h*row1)) are written at h_rgb + y*pitch, split
 * over n_threads (1..256) host threads.  Reads the blocks mjd_decode reads.
 * It is not a substitute for the device path: no call falls back to it. */
int mjd_decode_host(const mjd_frame* frame, const int16_t* h_coef, const uint16_t* h_qt, int upsample,
                    uint8_t* h_rgb, size_t pitch, uint32_t mcu_row0, uint32_t mcu_row1, int n_threads);

/* ---------------------------------------------------------------------
 * Decoder variants (paper Sec. 2 and Sec. 3 name libjpeg's AAN-based and
 * integer-or-float IDCTs; Sec. 4.2 decodes samplings other than 4:4:4 and
 * 4:2:2 the same way).  Full-size colour images decode in one launch of
 * the fused segment kernel for their sampling and IDCT method (no sample
 * planes in memory, no workspace).  Grayscale decodes in one launch that
 * writes its rows directly; scaled decodes use two launches: dequantise +
 * reduced IDCT into per-component sample planes in a caller workspace,
 * then upsampling + colour conversion.
 * IDCT methods:
 *   MJD_IDCT_ISLOW  LL&M in 13-bit fixed point (mjd_decode's arithmetic);
 *   MJD_IDCT_IFAST  the AAN flowgraph (transposed forward graph) in fixed
 *                   point: multipliers q * 2^6 / (s(u) s(v)) with
 *                   s(0) = 1, s(k) = sqrt(2) cos(k pi / 16), 9-bit
 *                   constants, truncating products; less accurate;
 *   MJD_IDCT_FLOAT  the same flowgraph in IEEE single precision.
 * Samplings: luma (h, v) of (1,1), (2,1), (1,2), (2,2) or (4,1), chroma
 * (1,1); fancy upsampling filters factors of 2 (Algorithm 1, vertical for
 * (1,2)) and replicates a factor of 4.  Grayscale: one component, blocks in
 * raster order, one output byte per pixel.
 * Scaled decoding (scale 2, 4, 8; islow only): each block's top-left N x N
 * coefficients (N = 8 / scale) through the N-point IDCT with the 8-point
 * normalisation, x(m,n) = 1/4 sum c(u) c(v) F(u,v) cos((2m+1)u pi/2N)
 * cos((2n+1)v pi/2N), in islow-style fixed point; the output is
 * ceil(W / scale) x ceil(H / scale), upsampled and converted at that size.
 * ------------------------------------------------------------------- */
enum { MJD_IDCT_ISLOW = 0, MJD_IDCT_IFAST = 1, MJD_IDCT_FLOAT = 2 };

typedef struct mjd_variant {
  mjd_frame frame;   /* as for mjd_decode; grayscale reads width, height, qsel[0] */
  uint32_t ncomp;    /* 3: YCbCr -> RGB8 (3 bytes per pixel); 1: grayscale (1 byte per pixel) */
  int32_t idct;      /* MJD_IDCT_* */
  int32_t upsample;  /* MJD_UPSAMPLE_* (unused for grayscale) */
  uint32_t scale;    /* output 1/scale of the image in each direction: 0 or 1 (full size), 2, 4 or 8 */
} mjd_variant;

/* Host only: validates `variant` and gives its geometry: the coefficient
 * layout (grayscale: 8x8 MCUs of one block), comp_w/comp_h at the output
 * scale (0 for absent components), and the workspace mjd_decode_variant
 * needs (0 for grayscale and for full-size colour images).  out and work_bytes
 * may be NULL.  MJD_EINVAL for bad fields, MJD_EUNSUPPORTED for other
 * samplings. */
int mjd_variant_geometry(const mjd_variant* variant, mjd_geometry* out, uint64_t* work_bytes);

/* Decodes a whole image.  d_coef: n_blocks * 64 int16 in MCU order,
 * 16-byte aligned (same numeric domain as mjd_decode); d_qt: uint16[4][64];
 * d_out: ceil(H / scale) rows of `pitch` bytes (pitch >= ncomp * ceil(W /
 * scale), < 2^31; < 2^24 for full-size colour images), only each row's
 * first ncomp * ceil(W / scale) bytes written; d_work: device workspace of
 * at least the size mjd_variant_geometry gives, 16-byte aligned, owned by
 * the caller, overwritten (may be NULL when that size is 0).  A full-size
 * colour image runs with the context's tuning (segment length, workgroup
 * count; the shape index only where the sampling's islow kernel is
 * mjd_decode's), which changes speed only.  Asynchronous on `stream`.
 * MJD_EINVAL for bad arguments, MJD_EDEVICE for launch failures. */
int mjd_decode_variant(mjd_ctx* ctx, const mjd_variant* variant, const int16_t* d_coef, const uint16_t* d_qt,
                       uint8_t* d_out, size_t pitch, void* d_work, uint64_t work_bytes, void* stream);

/* Heterogeneous decode of one bitstream (paper Sec. 5.2): the GPU decodes
 * the image's first MCU rows while host threads decode the rest, as a
 * partition (mjd_partition_rows) assigns them.  Owns pinned coefficient
 * staging, device buffers for the largest image, a stream and a pool of
 * host threads; calls on one decoder must not overlap (use one decoder per
 * calling thread). */
typedef struct mjd_hetero mjd_hetero;

/* Seconds spent in each part of one mjd_hetero_decode, on the host clock. */
typedef struct mjd_hetero_times {
  double huff_gpu_s; /* Huffman decoding of the rows the GPU needs (SPS: all rows) */
  double dispatch_s; /* enqueueing the GPU part: copies in, kernels, copies out */
  double huff_cpu_s; /* OVERLAP, PPS: Huffman decoding of the rows left for the CPU */
  double cpu_s;      /* mjd_decode_host of the CPU's rows */
  double gpu_s;      /* device time from the GPU part's first copy in to its last copy out */
  double total_s;    /* the whole call */
  uint32_t chunks;   /* GPU launches (one per chunk) */
  uint32_t cpu_rows; /* the CPU's rows in the end (PPS re-partitioning may change them) */
} mjd_hetero_times;

/* max_blocks / max_pixels: the largest image; n_threads (1..256) host
 * threads for Huffman decoding and the CPU rows (the caller's thread is one
 * of them).  When the process may run on at least n_threads CPUs, each
 * thread is pinned to a CPU of its own (the caller's thread only while a
 * decode runs, its affinity restored afterwards), so the host side runs on
 * as many distinct cores as the performance model was fitted with. */
int mjd_hetero_create(mjd_ctx* ctx, uint64_t max_blocks, uint64_t max_pixels, int n_threads, mjd_hetero** out);

/* How one image is shared. */
typedef struct mjd_hetero_plan {
  int scheme;              /* MJD_PART_SPS, MJD_PART_OVERLAP or MJD_PART_PPS */
  uint32_t cpu_rows;       /* 0, the height, or the height minus a multiple of the MCU height */
  uint32_t chunk_mcu_rows; /* PPS: MCU rows per GPU chunk (0: all the GPU's rows in one) */
  uint32_t pad;
  const struct mjd_model* model; /* PPS: re-partition before the last of two or more chunks with
                              mjd_repartition_rows (NULL: keep cpu_rows) */
  double huff_threads;     /* PPS re-partitioning: as for mjd_partition_rows */
} mjd_hetero_plan;

/* Decodes h_jpg into h_rgb (height rows of pitch bytes; pinned memory lets
 * the GPU rows arrive by DMA) as the plan shares it.  Returns when every
 * row is in h_rgb; times may be NULL.  Bit-exact with mjd_decode of the
 * whole image, whatever the plan.  MJD_EINVAL for null pointers, an unknown
 * scheme, an image above the decoder's capacity, pitch < 3 * width, or
 * cpu_rows off an MCU-row boundary; a bitstream's errors as mjd_parse. */
int mjd_hetero_decode(mjd_hetero* h, const uint8_t* h_jpg, size_t len, int upsample, const mjd_hetero_plan* plan,
                      uint8_t* h_rgb, size_t pitch, mjd_hetero_times* times);

/* Synchronise and free. */
void mjd_hetero_destroy(mjd_hetero* h);

/* One image of a batch: its frame, device buffers and output pitch, with
 * the same meaning and constraints as the arguments of mjd_decode (whole
 * image: MCU rows [0, mcus_y)). */
typedef struct mjd_job {
  mjd_frame frame;
  const int16_t* d_coef;
  const uint16_t* d_qt;
  uint8_t* d_rgb;
  size_t pitch;
} mjd_job;

/* A planned batch: device tables describing many images and the work queue
 * over them, owned by the library until mjd_batch_destroy. */
typedef struct mjd_batch mjd_batch;

/* Plan a batch of `n` images of any supported sizes and samplings, all
 * decoded with the same upsampling mode.  Validates every job (an invalid job
 * fails the whole call, naming the job), cuts every image into segments of
 * sub-tiles (the paper's horizontal chunks, Sec. 4.5, here also cut into MCU
 * columns) and uploads the per-image views and the segment queue, longest
 * segments first, to device memory (synchronous).  The launch shape follows
 * the context's tuning at the time of this call.  The device buffers named by
 * the jobs are only recorded, not accessed. */
int mjd_batch_create(mjd_ctx* ctx, const mjd_job* jobs, size_t n, int upsample, mjd_batch** out);

/* Enqueue the whole batch as ONE persistent kernel on `stream`: resident
 * workgroups pop segments from a device counter until the queue is empty;
 * the last workgroup rearms the counter.  use_graph != 0 launches it through
 * a hipGraph instantiated on first use and replayed afterwards.  Launches of
 * one batch must be serialised (one stream); each writes every job's output. */
int mjd_batch_launch(mjd_batch* batch, int use_graph, void* stream);

/* Segments in the queue, workgroups per launch and total pixels. */
int mjd_batch_info(const mjd_batch* batch, uint32_t* segments, uint32_t* workgroups, uint64_t* pixels);

/* Synchronise the device and free the batch's tables and graph. */
void mjd_batch_destroy(mjd_batch* batch);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * decode as mjd_batch_create + mjd_batch_launch(direct) + destroy, in one
 * call that allocates no device memory.  The batch tables (queue counters,
 * image views, segment queue) go into a fixed 4 MiB device array of the
 * library, one per GPU and held until the process ends, by one host-to-device
 * copy on `stream`, followed by the persistent kernel on `stream`.
 *   jobs, n, upsample: as for mjd_batch_create (host array, read during the
 *     call only); the jobs' device buffers must stay valid until the kernel
 *     has finished.
 * Returns MJD_EBUDGET (nothing enqueued) when the tables would exceed 4 MiB,
 * e.g. more than about 58000 images or 130000 segments.  Every call on one
 * GPU shares that array, which keeps the last call's contents: calls that
 * overlap on one GPU (different streams, or another context on the same
 * device) race, so they must be ordered by one stream or a synchronisation. */
int mjd_decode_batch_noalloc(mjd_ctx* ctx, const mjd_job* jobs, size_t n, int upsample, void* stream);

/* ---------------------------------------------------------------------
 * Host side: baseline JPEG bitstreams -> coefficient blocks.
 *
 * The paper keeps entropy decoding on the CPU because Huffman code words
 * have variable length, which makes it sequential (Sec. 1; Sec. 4.5).  Here
 * the restart intervals of the scan (DRI/RSTn, T.81 B.2.4.4 and F.2) are
 * independent, so several host threads decode them at once.  The frame
 * structure read here is the one the paper lists (Sec. 2): frame header with
 * the dimensions and sampling factors, quantisation tables, Huffman tables,
 * and the entropy-coded data.
 * ------------------------------------------------------------------- */

/* One Huffman table as a DHT segment defines it. */
typedef struct mjd_huffman {
  uint8_t bits[16];  /* number of codes of length 1..16 */
  uint8_t vals[256]; /* symbols in order of increasing code */
  uint32_t defined;  /* nonzero once a DHT segment defined the table */
} mjd_huffman;

/* Everything the entropy decoder needs about one baseline scan. */
typedef struct mjd_scan {
  mjd_frame frame;           /* frame header, in the form mjd_decode takes */
  uint32_t restart_interval; /* MCUs per restart interval (DRI); 0 = none */
  uint32_t n_intervals;      /* entropy-coded segments: ceil(MCUs / interval), or 1 */
  uint64_t data_offset;      /* byte offset of the first entropy-coded byte */
  uint64_t data_end;         /* byte offset of the EOI marker */
  uint8_t dc_sel[3];         /* DC Huffman table per component (0..3) */
  uint8_t ac_sel[3];         /* AC Huffman table per component (0..3) */
  uint8_t ncomp;             /* 3, or 1 for a grayscale frame (component 0 only, one block per MCU,
                                frame h/v 1x1; decode it with mjd_decode_variant, ncomp 1) */
  uint8_t reserved;
  mjd_huffman dc[4];
  mjd_huffman ac[4];
} mjd_scan;

/* Parse the markers of a baseline (SOF0/SOF1, 8-bit) JPEG held in host
 * memory: SOI, DQT, SOF, DHT, DRI, one SOS over the three components in
 * frame order (Ss=0, Se=63, Ah=Al=0), EOI; APPn and COM are skipped.
 *   h_qt: receives uint16[4][64] in natural order (tables the stream does
 *         not define are all ones).
 * Returns MJD_ECORRUPT for malformed or truncated streams (a 16-bit DQT
 * table, which T.81 B.2.4.1 allows only in 12-bit frames, included) and
 * MJD_EUNSUPPORTED for valid JPEG this library does not decode
 * (progressive, arithmetic, 12-bit, neither three components nor one,
 * sampling other than 4:4:4 / 4:2:2 / 4:2:0 and the variant samplings
 * h1v2 / 4:1:1, which only mjd_decode_variant decodes like grayscale; more
 * than one scan).  Reads only
 * [h_jpg, h_jpg + len). */
int mjd_parse(const uint8_t* h_jpg, size_t len, mjd_scan* scan, uint16_t h_qt[4][64]);

/* Locate the restart intervals: h_offsets[i] (i < n_intervals) receives
 * the byte offset of interval i's first entropy-coded byte, and
 * h_offsets[n_intervals] the offset just past the EOI marker, so interval
 * i's data ends 2 bytes (its RSTn or EOI marker) before h_offsets[i + 1],
 * not counting 0xFF fill bytes.  h_offsets holds n_intervals + 1 entries.
 * MJD_ECORRUPT if the RSTn markers are missing, out of sequence or too
 * many. */
int mjd_restart_index(const uint8_t* h_jpg, size_t len, const mjd_scan* scan, uint64_t* h_offsets);

/* Huffman-decode MCU rows [mcu_row0, mcu_row1) into h_coef, which holds the
 * whole image's n_blocks * 64 int16 in the MCU order mjd_decode reads
 * (natural order inside a block, DC prediction applied).  Only the blocks
 * of those rows are written.  Restart intervals that cover the rows are
 * decoded by up to n_threads threads (created for this call; 1 = the
 * calling thread only); an interval that starts before mcu_row0 is decoded
 * from its start and its earlier MCUs are discarded.  Without restart
 * markers the whole scan is one interval.  h_offsets is the output of
 * mjd_restart_index, or NULL to have it computed here.  MJD_ECORRUPT for
 * invalid codes, coefficient runs past the end of a block, or an interval
 * that needs more bits than its data holds.  Huffman data cannot be
 * resynchronised inside an interval (paper Sec. 1: no code word marks a
 * block boundary), but the next restart marker is a resync point: every
 * other interval is still decoded, the blocks of a corrupt interval's MCUs
 * inside the rows are set to zero (mid-grey after the back half), and the
 * message names the lowest-numbered corrupt interval.  Memory-safe for any
 * input bytes. */
int mjd_entropy_decode(const uint8_t* h_jpg, size_t len, const mjd_scan* scan, const uint64_t* h_offsets,
                       int16_t* h_coef, uint32_t mcu_row0, uint32_t mcu_row1, int n_threads);

/* ---------------------------------------------------------------------
 * GPU entropy decoding of many baseline scans.  Restart intervals restart
 * the bit stream and the DC predictions (ITU-T T.81 restart markers), so
 * each one decodes on its own: one GPU lane decodes one interval.  This
 * moves the part the paper leaves on the CPU (Sec. 1: variable-length code
 * words) onto the device whenever a stream has restart markers.  A stream
 * without them is one interval and decodes on one lane (correct but slow).
 * ------------------------------------------------------------------- */

/* One scan to decode on the device. */
typedef struct mjd_entropy_job {
  const mjd_scan* scan;      /* host: from mjd_parse; read at create time */
  const uint64_t* h_offsets; /* host: from mjd_restart_index (n_intervals + 1
                                entries); read at create time */
  const uint8_t* d_jpg;      /* device, 16-byte aligned: the whole stream,
                                bytes [0, len); the buffer must be readable
                                up to len rounded up to a multiple of 16 */
  uint64_t len;              /* bytes of the stream at d_jpg */
  int16_t* d_coef;           /* device, 16-byte aligned: n_blocks * 64 int16
                                in the MCU order mjd_decode reads (natural
                                order inside a block, DC prediction applied);
                                every block is written */
} mjd_entropy_job;

/* Planned GPU entropy decoding of many scans, owned by the library until
 * mjd_entropy_batch_destroy. */
typedef struct mjd_entropy_batch mjd_entropy_batch;

/* Check the jobs and plan them: build each scan's Huffman tables in device
 * form, list the restart intervals (byte ranges from h_offsets, which must
 * be increasing and inside [0, len)) and upload the tables (synchronous).
 * An invalid job fails the whole call, naming the job.  The device buffers
 * are only recorded, not accessed. */
int mjd_entropy_batch_create(mjd_ctx* ctx, const mjd_entropy_job* jobs, size_t n, mjd_entropy_batch** out);

/* Enqueue the decoding of every job on `stream`: one persistent kernel whose
 * workgroups take up to 256 intervals of one job at a time.  Launches of one
 * batch must be serialised (one stream).  Reads only the first len bytes of
 * each job's stream, rounded up to 16, and writes only its coefficient
 * blocks. */
int mjd_entropy_batch_launch(mjd_entropy_batch* batch, void* stream);

/* Synchronise the device and check the last launch: MJD_OK, or
 * MJD_ECORRUPT naming the first job and restart interval that held an
 * invalid Huffman code, a coefficient run past the end of a block, or too
 * few bits for its MCUs (*bad_job receives the job, else -1; may be NULL).
 * The blocks of a corrupt interval are then unspecified. */
int mjd_entropy_batch_status(mjd_entropy_batch* batch, int64_t* bad_job);

/* Restart intervals in the batch, workgroups per launch and stream bytes. */
int mjd_entropy_batch_info(const mjd_entropy_batch* batch, uint32_t* intervals, uint32_t* workgroups,
                           uint64_t* bytes);

/* Synchronise the device and free the batch's tables. */
void mjd_entropy_batch_destroy(mjd_entropy_batch* batch);

/* ---------------------------------------------------------------------
 * Pipelined end-to-end decode: bitstreams in host memory -> RGB8 in host
 * memory.  The paper's pipelined GPU mode (Sec. 4.5, Fig. 6) cuts an image
 * into horizontal chunks so that the entropy decoding of chunk i+1 on the
 * CPU overlaps the transfer and the kernels of chunk i on the GPU.  Here the
 * chunks are MCU-row bands; host worker threads decode the restart
 * intervals of each band into pinned buffers, and each finished band goes
 * host->device on one HIP stream, through the fused kernel on a second and
 * back device->host on a third, while the workers move on to the next band
 * and the next images.
 * ------------------------------------------------------------------- */

typedef struct mjd_pipeline mjd_pipeline;

enum {
  /* Host entropy decoding only, into the pinned slots; nothing is sent to
   * the device.  Its wall time is the entropy-bound limit of the pipeline. */
  MJD_PIPELINE_ENTROPY_ONLY = 1
};

typedef struct mjd_pipeline_config {
  uint32_t n_threads;     /* entropy worker threads (>= 1) */
  uint32_t n_slots;       /* images in flight (>= 2): pinned + device buffers each */
  uint32_t band_mcu_rows; /* MCU rows per band; 0 = about 8 bands per image */
  uint32_t upsample;      /* MJD_UPSAMPLE_* */
  uint64_t max_blocks;    /* coefficient blocks of the largest image a slot holds */
  uint64_t max_pixels;    /* width * height of the largest image a slot holds */
} mjd_pipeline_config;

/* Totals of one mjd_pipeline_run.  Stage times are sums over bands of
 * HIP event intervals (the stages overlap, so they do not add up to the
 * wall time); entropy_ms sums the worker threads' decoding time. */
typedef struct mjd_pipeline_stats {
  double wall_ms;
  double entropy_ms;
  double parse_ms;
  double h2d_ms;
  double kernel_ms;
  double d2h_ms;
  uint64_t images;
  uint64_t pixels;
  uint64_t bitstream_bytes;
  uint64_t bands;
} mjd_pipeline_stats;

/* Create the worker threads, n_slots pinned host coefficient buffers of
 * max_blocks * 128 bytes, the matching device coefficient and RGB buffers
 * (max_pixels * 3 bytes) and three streams on the context's device. */
int mjd_pipeline_create(mjd_ctx* ctx, const mjd_pipeline_config* cfg, mjd_pipeline** out);

/* Decode n bitstreams end to end, in order: image i is parsed (mjd_parse),
 * its restart intervals are decoded on the workers, and its RGB8 rows land
 * at h_rgb[i] + y * pitches[i] (pitch >= 3 * width).  Returns when every
 * output is in host memory.  h_rgb buffers should be pinned
 * (hipHostMalloc) for the device->host copies to overlap; outputs may share
 * a buffer, in which case the last image written wins.  flags:
 * MJD_PIPELINE_ENTROPY_ONLY or 0.  An image larger than the slots gives
 * MJD_EBUDGET, a corrupt one MJD_ECORRUPT (naming the image); the run stops
 * at the first failure after draining the work in flight.  stats may be
 * NULL.  One run at a time per pipeline. */
int mjd_pipeline_run(mjd_pipeline* pipe, size_t n, const uint8_t* const* h_jpgs, const size_t* lens,
                     uint8_t* const* h_rgb, const size_t* pitches, uint32_t flags, mjd_pipeline_stats* stats);

/* Stop the workers and free every buffer, stream and event. */
void mjd_pipeline_destroy(mjd_pipeline* pipe);

/* ---------------------------------------------------------------------
 * Performance model (paper Sec. 5.1).  Decode times are predicted from
 * closed forms fitted once, off-line, to times measured on this machine:
 *   d = file bytes / (w * h)                           (Eq. 3)
 *   T_huff(w, h, d) = T_huff_per_pixel(d) * w * h      (Eq. 4)
 *   P_gpu(w, h) = O_w(w, h) + T_kernel(w, h) + O_r(w, h)
 *                                (host->device, kernel, device->host)
 *   T_total = T_huff + P_gpu
 * Each closed form is a polynomial of degree at most 7: in d for the
 * Huffman rate, in the scaled dimensions (a, b) = (w / 1024, h / 1024) for
 * the GPU parts.  It is fitted by least squares; its degree is the one of
 * least Akaike information criterion; it is evaluated in Horner form.
 * Host code only: these calls touch no device.
 * ------------------------------------------------------------------- */
#define MJD_POLY_MAX_DEGREE 7
#define MJD_POLY2_TERMS 36 /* (7 + 1) * (7 + 2) / 2 */

/* p(x) = sum over i <= degree of c[i] * x^i. */
typedef struct mjd_poly1 {
  int32_t degree;
  int32_t pad;
  double c[MJD_POLY_MAX_DEGREE + 1];
} mjd_poly1;

/* p(a, b) = sum over i + j <= degree of c[t(i, j)] * a^i * b^j, with the
 * terms grouped by the power of a: t(i, j) = i * (2 * degree + 3 - i) / 2 + j. */
typedef struct mjd_poly2 {
  int32_t degree;
  int32_t pad;
  double c[MJD_POLY2_TERMS];
} mjd_poly2;

/* Least-squares fits of every degree 0..max_degree whose k terms are fewer
 * than the n samples; keeps the one of least AIC = n * ln(RSS / n) + 2k.
 * A residual sum below 1e-24 of sum(y^2) counts as that floor, so that
 * among exact fits the one with fewest terms wins.  *aic receives the kept
 * fit's AIC (may be NULL).  MJD_EINVAL for null pointers, max_degree
 * outside 0..7 or fewer than 2 samples; MJD_EUNSUPPORTED when no degree
 * could be fitted (every design matrix rank-deficient). */
int mjd_poly1_fit(const double* x, const double* y, size_t n, int max_degree, mjd_poly1* out, double* aic);
int mjd_poly2_fit(const double* a, const double* b, const double* y, size_t n, int max_degree, mjd_poly2* out,
                  double* aic);

/* Horner evaluation (the paper's form for run-time prediction). */
double mjd_poly1_eval(const mjd_poly1* p, double x);
double mjd_poly2_eval(const mjd_poly2* p, double a, double b);

/* The fitted model: Huffman seconds per pixel against d (bytes per
 * pixel), and the three GPU parts in seconds against (w / 1024, h / 1024);
 * for CPU-GPU partitioning also the back half on host cores (P_cpu) and the
 * host's time to enqueue the GPU part (T_dispatch), against (w / 1024,
 * rows / 1024). */
typedef struct mjd_model {
  mjd_poly1 huff_per_pixel;
  mjd_poly2 o_w, t_kernel, o_r;
  mjd_poly2 p_cpu, t_dispatch;
} mjd_model;

/* One prediction, in seconds (d in bytes per pixel); total = t_huff + p_gpu. */
typedef struct mjd_prediction {
  double d, t_huff, o_w, t_kernel, o_r, p_gpu, total, p_cpu, t_dispatch;
} mjd_prediction;

/* Evaluates the model for one image (Eqs. 3-4 and the sums above).
 * MJD_EINVAL for null pointers or a zero dimension. */
int mjd_model_predict(const mjd_model* model, uint32_t width, uint32_t height, uint64_t file_bytes,
                      mjd_prediction* out);

/* CPU-GPU partitioning of one image (paper Sec. 5.2).  The GPU decodes the
 * image's first rows and the CPU the last x rows, x chosen so that both
 * sides finish together (f(x) = 0), by Newton's method on the model's
 * polynomials (from h/2, kept inside [0, h], until a step no longer reduces
 * |f|), then rounded so that the GPU keeps whole MCU rows.  Huffman terms
 * are T_huff(w, rows, d) = huff_per_pixel(d) * w * rows / huff_threads.
 *   SPS (simple, Eqs. 8-10): Huffman decoding of the whole image first, then
 *     f(x) = T_dispatch(w, h-x) + P_cpu(w, x) - P_gpu(w, h-x).
 *   OVERLAP (Fig. 7b, Eqs. 12-13): Huffman decoding of the GPU's rows, the
 *     dispatch, then the CPU decodes its own rows' Huffman data while the
 *     GPU works:
 *     f(x) = T_dispatch(w, h-x) + T_huff(w, x, d) + P_cpu(w, x) - P_gpu(w, h-x).
 *   PPS (pipelined, Eqs. 14-15): the GPU's rows go in chunks, each launched
 *     as soon as its Huffman data is decoded; after the first chunk of c
 *     rows the CPU decodes every remaining row's Huffman data, then its own
 *     rows:
 *     f(x) = T_huff(w, h-c, d) + P_cpu(w, x) + T_dispatch(w, h-x) - P_gpu(w, h-x),
 *     with c = min(chunk_rows, h-x).
 * huff_threads: the speed-up of the host Huffman decoder over the model's
 * one-thread rate (restart intervals decode in parallel); >= 1.
 * chunk_rows: PPS only, the GPU chunk's height in rows (> 0).
 * MJD_EINVAL for null pointers, a zero dimension, an MCU height other than
 * 8 or 16, an unknown scheme, huff_threads < 1 or PPS without chunk_rows. */
enum { MJD_PART_SPS = 0, MJD_PART_OVERLAP = 1, MJD_PART_PPS = 2 };

typedef struct mjd_partition {
  uint32_t cpu_rows;   /* the CPU's rows: rows - (GPU's whole MCU rows) * mcu_h */
  uint32_t iterations; /* Newton steps taken */
  double x;            /* the unrounded balance point in rows (0 or all rows when f keeps one sign) */
  double t_cpu, t_gpu; /* predicted seconds of both sides at cpu_rows, after the common Huffman prefix */
} mjd_partition;

int mjd_partition_rows(const mjd_model* model, int scheme, uint32_t width, uint32_t height, uint32_t mcu_h,
                       uint64_t file_bytes, double huff_threads, uint32_t chunk_rows, mjd_partition* out);

/* PPS re-partitioning before the GPU's last chunk (paper Sec. 5.2, Eqs.
 * 16-17).  rows_left: the image's rows from the first row not yet given to
 * the GPU to the bottom (the last chunk and the CPU's rows; the split is on
 * an MCU-row boundary of these rows); huff_rows_left: the rows whose Huffman
 * data is still undecoded; huff_done_s: the measured seconds of Huffman
 * decoding so far; gpu_busy_s: the estimated device time still owed to the
 * earlier chunks.  The density of the undecoded rows is
 *   d' = (max(0, E - huff_done_s) / E) / (huff_rows_left / h) * d,
 * E = T_huff(w, h, d) the estimate for the whole image, and the split of
 * rows_left solves
 *   f(x') = T_dispatch(w, r-x') + T_huff(w, huff_rows_left, d') + P_cpu(w, x')
 *           - P_gpu(w, r-x') - gpu_busy_s,   r = rows_left.
 * out->cpu_rows is x' rounded (the CPU's rows, at the bottom of the image).
 * MJD_EINVAL for null pointers, bad dimensions, rows_left outside
 * 1..height, negative times or huff_threads < 1. */
int mjd_repartition_rows(const mjd_model* model, uint32_t width, uint32_t height, uint32_t rows_left, uint32_t mcu_h,
                         uint64_t file_bytes, double huff_threads, uint32_t huff_rows_left, double huff_done_s,
                         double gpu_busy_s, mjd_partition* out);

/* ---------------------------------------------------------------------
 * Serving: a request loop that decodes images of different sizes as they
 * arrive.  Requests carry quantised coefficients in host memory (the
 * paper's input, Sec. 7) and receive RGB8 in host memory (or in device
 * memory, for consumers on the GPU).  The server keeps
 * one device arena of `budget_bytes` for the coefficient and RGB buffers of
 * admitted requests (the paper's whole-image buffers, Sec. 4); a request is
 * admitted, in arrival order, once it has arrived and its buffers fit.
 * Continuous batching: every request admitted while earlier batches are on
 * the device is copied host->device at once and joins the next persistent
 * batch launch; results go device->host on their own stream and free the
 * arena as they complete.  The server thread uses the context (its tuning
 * and device) while it runs: do not change the context's tuning meanwhile.
 * ------------------------------------------------------------------- */

typedef struct mjd_server mjd_server;

enum {
  MJD_SERVE_CONTINUOUS = 0, /* continuous batching (above) */
  MJD_SERVE_SYNC = 1        /* one request at a time: copy, decode, copy back, synchronise */
};

typedef struct mjd_server_config {
  uint64_t budget_bytes; /* device arena for coefficient + RGB buffers (e.g. 16 GiB) */
  uint32_t upsample;     /* MJD_UPSAMPLE_* */
  uint32_t mode;         /* MJD_SERVE_* */
  uint32_t max_batch;    /* requests per batch launch, 1..4096 */
  uint32_t max_inflight; /* batch launches on the device at once, 1..8 */
  const mjd_model* model; /* optional (NULL: none); copied at create */
  double max_batch_s;     /* with a model and > 0: a batch admits requests
                             while the sum of their predicted GPU times
                             (O_w + T_kernel + O_r) stays within this many
                             seconds; its first request always */
} mjd_server_config;

/* One decode request.  All buffers belong to the caller and must stay valid
 * until the request is done; h_coef/h_qt are read, h_rgb written, by device
 * copies (pinned memory lets them overlap).  Exactly one of h_rgb and d_rgb
 * is set: with d_rgb (device memory on the server's device, for consumers
 * that stay on the GPU) the batch kernel writes the rows there itself, the
 * arena holds no RGB buffer for the request and nothing is copied back. */
typedef struct mjd_request {
  mjd_frame frame;
  const int16_t* h_coef; /* n_blocks * 64 int16, MCU order (as mjd_decode) */
  const uint16_t* h_qt;  /* uint16[4][64] */
  uint8_t* h_rgb;        /* height rows of pitch bytes in host memory, or NULL */
  uint64_t pitch;        /* >= 3 * width */
  uint64_t arrival_ns;   /* on the server clock (mjd_server_now_ns); earlier than now = arrived */
  uint8_t* d_rgb;        /* height rows of pitch bytes in device memory, or NULL */
} mjd_request;

/* Server-clock timestamps of one request (0 while a stage has not happened). */
typedef struct mjd_request_times {
  uint64_t arrival_ns;
  uint64_t admit_ns;   /* buffers allocated, host->device copy enqueued */
  uint64_t launch_ns;  /* its batch (or its decode, in sync mode) enqueued */
  uint64_t done_ns;    /* RGB8 in h_rgb, or written to d_rgb (observed by the server) */
  int32_t status;      /* MJD_OK, or why it failed */
  uint32_t batch;      /* number of requests in its batch launch */
} mjd_request_times;

/* Allocate the arena, batch tables and streams on the context's device and
 * start the server thread.  Its clock starts at 0 here. */
int mjd_server_create(mjd_ctx* ctx, const mjd_server_config* cfg, mjd_server** out);
/* Nanoseconds on the server clock. */
uint64_t mjd_server_now_ns(const mjd_server* srv);
/* Queue a request (thread-safe); *id numbers requests 0, 1, 2, ... in
 * submission order, which is the admission order.  Validation happens here:
 * MJD_EBUDGET if the request's buffers can never fit in the arena; arrival
 * times must not decrease from one request to the next. */
int mjd_server_submit(mjd_server* srv, const mjd_request* req, uint64_t* id);
/* Block until request `id` is done; fills its timestamps.  Returns its
 * status.  Records of finished requests are kept until mjd_server_destroy. */
int mjd_server_wait(mjd_server* srv, uint64_t id, mjd_request_times* times);
/* Block until every submitted request is done. */
int mjd_server_drain(mjd_server* srv);
/* Drain, stop the server thread and free everything. */
void mjd_server_destroy(mjd_server* srv);

/* Device-to-device streaming copy of `bytes` bytes (a multiple of 16; both
 * pointers 16-byte aligned), enqueued on `stream`.  It is the bandwidth
 * reference for the decoder: a plain read+write stream at the rate this
 * device sustains, used as the denominator check of the roofline and to
 * calibrate memory-traffic counters. */
int mjd_copy(mjd_ctx* ctx, void* d_dst, const void* d_src, size_t bytes, void* stream);

/* Thread-local description of the last error on this thread ("" if none). */
const char* mjd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MJD_H */
