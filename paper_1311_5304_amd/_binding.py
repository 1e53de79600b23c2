"""ctypes binding of libmjd.so: the C ABI in include/mjd.h, with the same names.

Argument marshalling only.  Device buffers are passed as torch tensors (their
data_ptr()) or as raw integer addresses; streams as torch.cuda.Stream, a raw
hipStream_t integer, or None for the current torch stream.  Nothing here
computes any part of the decode; if the library is missing, importing a
function raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libmjd.so")

MJD_OK = 0
MJD_POLY_MAX_DEGREE = 7
MJD_IDCT_ISLOW = 0
MJD_IDCT_IFAST = 1
MJD_IDCT_FLOAT = 2
IDCT = {"islow": MJD_IDCT_ISLOW, "ifast": MJD_IDCT_IFAST, "float": MJD_IDCT_FLOAT}
MJD_PART_SPS = 0
MJD_PART_OVERLAP = 1
MJD_PART_PPS = 2
MJD_EINVAL = -1
MJD_EUNSUPPORTED = -2
MJD_ENOMEM = -3
MJD_EDEVICE = -4
MJD_ECORRUPT = -5
MJD_EBUDGET = -6
STATUS_NAMES = {0: "MJD_OK", -1: "MJD_EINVAL", -2: "MJD_EUNSUPPORTED", -3: "MJD_ENOMEM",
                -4: "MJD_EDEVICE", -5: "MJD_ECORRUPT", -6: "MJD_EBUDGET"}

MJD_UPSAMPLE_SIMPLE = 0
MJD_UPSAMPLE_FANCY = 1


class MjdError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


class mjd_frame(ctypes.Structure):
    _fields_ = [("width", ctypes.c_uint32), ("height", ctypes.c_uint32),
                ("h", ctypes.c_uint8 * 3), ("v", ctypes.c_uint8 * 3),
                ("qsel", ctypes.c_uint8 * 3), ("reserved", ctypes.c_uint8)]


class mjd_geometry(ctypes.Structure):
    _fields_ = [("mcu_w", ctypes.c_uint32), ("mcu_h", ctypes.c_uint32),
                ("mcus_x", ctypes.c_uint32), ("mcus_y", ctypes.c_uint32),
                ("blocks_per_mcu", ctypes.c_uint32),
                ("comp_w", ctypes.c_uint32 * 3), ("comp_h", ctypes.c_uint32 * 3),
                ("n_blocks", ctypes.c_uint64)]


class mjd_tuning(ctypes.Structure):
    _fields_ = [("seg_subtiles", ctypes.c_uint32), ("workgroups", ctypes.c_uint32), ("shape", ctypes.c_uint32)]


class mjd_shape(ctypes.Structure):
    _fields_ = [("mcus_x", ctypes.c_uint32), ("mcus_y", ctypes.c_uint32), ("threads", ctypes.c_uint32),
                ("lds_bytes", ctypes.c_uint32), ("resident_per_cu", ctypes.c_uint32), ("cu_count", ctypes.c_uint32)]


class mjd_job(ctypes.Structure):
    _fields_ = [("frame", mjd_frame), ("d_coef", ctypes.c_void_p), ("d_qt", ctypes.c_void_p),
                ("d_rgb", ctypes.c_void_p), ("pitch", ctypes.c_size_t)]


class mjd_huffman(ctypes.Structure):
    _fields_ = [("bits", ctypes.c_uint8 * 16), ("vals", ctypes.c_uint8 * 256), ("defined", ctypes.c_uint32)]


class mjd_scan(ctypes.Structure):
    _fields_ = [("frame", mjd_frame), ("restart_interval", ctypes.c_uint32), ("n_intervals", ctypes.c_uint32),
                ("data_offset", ctypes.c_uint64), ("data_end", ctypes.c_uint64),
                ("dc_sel", ctypes.c_uint8 * 3), ("ac_sel", ctypes.c_uint8 * 3), ("ncomp", ctypes.c_uint8),
                ("reserved", ctypes.c_uint8),
                ("dc", mjd_huffman * 4), ("ac", mjd_huffman * 4)]


class mjd_entropy_job(ctypes.Structure):
    _fields_ = [("scan", ctypes.POINTER(mjd_scan)), ("h_offsets", ctypes.c_void_p), ("d_jpg", ctypes.c_void_p),
                ("len", ctypes.c_uint64), ("d_coef", ctypes.c_void_p)]


class mjd_poly1(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("pad", ctypes.c_int32), ("c", ctypes.c_double * 8)]


class mjd_poly2(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("pad", ctypes.c_int32), ("c", ctypes.c_double * 36)]


class mjd_model(ctypes.Structure):
    _fields_ = [("huff_per_pixel", mjd_poly1), ("o_w", mjd_poly2), ("t_kernel", mjd_poly2), ("o_r", mjd_poly2),
                ("p_cpu", mjd_poly2), ("t_dispatch", mjd_poly2)]


class mjd_prediction(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("d", "t_huff", "o_w", "t_kernel", "o_r", "p_gpu", "total",
                                               "p_cpu", "t_dispatch")]


class mjd_partition(ctypes.Structure):
    _fields_ = [("cpu_rows", ctypes.c_uint32), ("iterations", ctypes.c_uint32), ("x", ctypes.c_double),
                ("t_cpu", ctypes.c_double), ("t_gpu", ctypes.c_double)]


class mjd_hetero_times(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("huff_gpu_s", "dispatch_s", "huff_cpu_s", "cpu_s", "gpu_s",
                                               "total_s")] + [("chunks", ctypes.c_uint32),
                                                              ("cpu_rows", ctypes.c_uint32)]


class mjd_hetero_plan(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("cpu_rows", ctypes.c_uint32), ("chunk_mcu_rows", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("model", ctypes.c_void_p), ("huff_threads", ctypes.c_double)]


class mjd_variant(ctypes.Structure):
    _fields_ = [("frame", mjd_frame), ("ncomp", ctypes.c_uint32), ("idct", ctypes.c_int32),
                ("upsample", ctypes.c_int32), ("scale", ctypes.c_uint32)]


class mjd_pipeline_config(ctypes.Structure):
    _fields_ = [("n_threads", ctypes.c_uint32), ("n_slots", ctypes.c_uint32), ("band_mcu_rows", ctypes.c_uint32),
                ("upsample", ctypes.c_uint32), ("max_blocks", ctypes.c_uint64), ("max_pixels", ctypes.c_uint64)]


class mjd_pipeline_stats(ctypes.Structure):
    _fields_ = [("wall_ms", ctypes.c_double), ("entropy_ms", ctypes.c_double), ("parse_ms", ctypes.c_double),
                ("h2d_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double), ("d2h_ms", ctypes.c_double),
                ("images", ctypes.c_uint64), ("pixels", ctypes.c_uint64), ("bitstream_bytes", ctypes.c_uint64),
                ("bands", ctypes.c_uint64)]


MJD_PIPELINE_ENTROPY_ONLY = 1
MJD_SERVE_CONTINUOUS = 0
MJD_SERVE_SYNC = 1


class mjd_server_config(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("upsample", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("max_batch", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32), ("model", ctypes.c_void_p),
                ("max_batch_s", ctypes.c_double)]


class mjd_request(ctypes.Structure):
    _fields_ = [("frame", mjd_frame), ("h_coef", ctypes.c_void_p), ("h_qt", ctypes.c_void_p),
                ("h_rgb", ctypes.c_void_p), ("pitch", ctypes.c_uint64), ("arrival_ns", ctypes.c_uint64),
                ("d_rgb", ctypes.c_void_p)]


class mjd_request_times(ctypes.Structure):
    _fields_ = [("arrival_ns", ctypes.c_uint64), ("admit_ns", ctypes.c_uint64), ("launch_ns", ctypes.c_uint64),
                ("done_ns", ctypes.c_uint64), ("status", ctypes.c_int32), ("batch", ctypes.c_uint32)]

_lib = None


def lib() -> ctypes.CDLL:
    """Load libmjd.so (built in-tree by paper_1311_5304_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1311_5304_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_size_t
        L.mjd_ctx_create.argtypes = [ctypes.POINTER(vp), i32]
        L.mjd_ctx_create.restype = i32
        L.mjd_ctx_destroy.argtypes = [vp]
        L.mjd_ctx_destroy.restype = None
        L.mjd_geometry_of.argtypes = [ctypes.POINTER(mjd_frame), ctypes.POINTER(mjd_geometry)]
        L.mjd_geometry_of.restype = i32
        L.mjd_decode.argtypes = [vp, ctypes.POINTER(mjd_frame), vp, vp, i32, vp, sz, u32, u32, vp]
        L.mjd_decode.restype = i32
        L.mjd_ctx_set_tuning.argtypes = [vp, ctypes.POINTER(mjd_tuning)]
        L.mjd_ctx_set_tuning.restype = i32
        L.mjd_ctx_get_tuning.argtypes = [vp, ctypes.POINTER(mjd_tuning)]
        L.mjd_ctx_get_tuning.restype = i32
        L.mjd_shape_count.argtypes = [u32, u32, i32, ctypes.POINTER(u32)]
        L.mjd_shape_count.restype = i32
        L.mjd_shape_info.argtypes = [vp, u32, u32, i32, u32, ctypes.POINTER(mjd_shape)]
        L.mjd_shape_info.restype = i32
        L.mjd_batch_create.argtypes = [vp, ctypes.POINTER(mjd_job), sz, i32, ctypes.POINTER(vp)]
        L.mjd_batch_create.restype = i32
        L.mjd_batch_launch.argtypes = [vp, i32, vp]
        L.mjd_batch_launch.restype = i32
        L.mjd_batch_info.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(ctypes.c_uint64)]
        L.mjd_batch_info.restype = i32
        L.mjd_decode_batch_noalloc.argtypes = [vp, ctypes.POINTER(mjd_job), sz, i32, vp]
        L.mjd_decode_batch_noalloc.restype = i32
        L.mjd_batch_destroy.argtypes = [vp]
        L.mjd_batch_destroy.restype = None
        L.mjd_parse.argtypes = [vp, sz, ctypes.POINTER(mjd_scan), vp]
        L.mjd_parse.restype = i32
        L.mjd_restart_index.argtypes = [vp, sz, ctypes.POINTER(mjd_scan), vp]
        L.mjd_restart_index.restype = i32
        L.mjd_entropy_decode.argtypes = [vp, sz, ctypes.POINTER(mjd_scan), vp, vp, u32, u32, i32]
        L.mjd_entropy_decode.restype = i32
        L.mjd_entropy_batch_create.argtypes = [vp, ctypes.POINTER(mjd_entropy_job), sz, ctypes.POINTER(vp)]
        L.mjd_entropy_batch_create.restype = i32
        L.mjd_entropy_batch_launch.argtypes = [vp, vp]
        L.mjd_entropy_batch_launch.restype = i32
        L.mjd_entropy_batch_status.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        L.mjd_entropy_batch_status.restype = i32
        L.mjd_entropy_batch_info.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32),
                                             ctypes.POINTER(ctypes.c_uint64)]
        L.mjd_entropy_batch_info.restype = i32
        L.mjd_entropy_batch_destroy.argtypes = [vp]
        L.mjd_entropy_batch_destroy.restype = None
        L.mjd_decode_host.argtypes = [ctypes.POINTER(mjd_frame), vp, vp, i32, vp, sz, u32, u32, i32]
        L.mjd_decode_host.restype = i32
        dp = ctypes.POINTER(ctypes.c_double)
        L.mjd_poly1_fit.argtypes = [dp, dp, sz, i32, ctypes.POINTER(mjd_poly1), dp]
        L.mjd_poly1_fit.restype = i32
        L.mjd_poly2_fit.argtypes = [dp, dp, dp, sz, i32, ctypes.POINTER(mjd_poly2), dp]
        L.mjd_poly2_fit.restype = i32
        L.mjd_poly1_eval.argtypes = [ctypes.POINTER(mjd_poly1), ctypes.c_double]
        L.mjd_poly1_eval.restype = ctypes.c_double
        L.mjd_poly2_eval.argtypes = [ctypes.POINTER(mjd_poly2), ctypes.c_double, ctypes.c_double]
        L.mjd_poly2_eval.restype = ctypes.c_double
        L.mjd_model_predict.argtypes = [ctypes.POINTER(mjd_model), u32, u32, ctypes.c_uint64,
                                        ctypes.POINTER(mjd_prediction)]
        L.mjd_model_predict.restype = i32
        L.mjd_partition_rows.argtypes = [ctypes.POINTER(mjd_model), i32, u32, u32, u32, ctypes.c_uint64,
                                         ctypes.c_double, u32, ctypes.POINTER(mjd_partition)]
        L.mjd_partition_rows.restype = i32
        L.mjd_repartition_rows.argtypes = [ctypes.POINTER(mjd_model), u32, u32, u32, u32, ctypes.c_uint64,
                                           ctypes.c_double, u32, ctypes.c_double, ctypes.c_double,
                                           ctypes.POINTER(mjd_partition)]
        L.mjd_repartition_rows.restype = i32
        L.mjd_variant_geometry.argtypes = [ctypes.POINTER(mjd_variant), ctypes.POINTER(mjd_geometry),
                                           ctypes.POINTER(ctypes.c_uint64)]
        L.mjd_variant_geometry.restype = i32
        L.mjd_decode_variant.argtypes = [vp, ctypes.POINTER(mjd_variant), vp, vp, vp, sz, vp, ctypes.c_uint64, vp]
        L.mjd_decode_variant.restype = i32
        L.mjd_hetero_create.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint64, i32, ctypes.POINTER(vp)]
        L.mjd_hetero_create.restype = i32
        L.mjd_hetero_decode.argtypes = [vp, vp, sz, i32, ctypes.POINTER(mjd_hetero_plan), vp, sz,
                                        ctypes.POINTER(mjd_hetero_times)]
        L.mjd_hetero_decode.restype = i32
        L.mjd_hetero_destroy.argtypes = [vp]
        L.mjd_hetero_destroy.restype = None
        L.mjd_pipeline_create.argtypes = [vp, ctypes.POINTER(mjd_pipeline_config), ctypes.POINTER(vp)]
        L.mjd_pipeline_create.restype = i32
        L.mjd_pipeline_run.argtypes = [vp, sz, vp, vp, vp, vp, u32, ctypes.POINTER(mjd_pipeline_stats)]
        L.mjd_pipeline_run.restype = i32
        L.mjd_pipeline_destroy.argtypes = [vp]
        L.mjd_pipeline_destroy.restype = None
        L.mjd_server_create.argtypes = [vp, ctypes.POINTER(mjd_server_config), ctypes.POINTER(vp)]
        L.mjd_server_create.restype = i32
        L.mjd_server_now_ns.argtypes = [vp]
        L.mjd_server_now_ns.restype = ctypes.c_uint64
        L.mjd_server_submit.argtypes = [vp, ctypes.POINTER(mjd_request), ctypes.POINTER(ctypes.c_uint64)]
        L.mjd_server_submit.restype = i32
        L.mjd_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(mjd_request_times)]
        L.mjd_server_wait.restype = i32
        L.mjd_server_drain.argtypes = [vp]
        L.mjd_server_drain.restype = i32
        L.mjd_server_destroy.argtypes = [vp]
        L.mjd_server_destroy.restype = None
        L.mjd_copy.argtypes = [vp, vp, vp, sz, vp]
        L.mjd_copy.restype = i32
        L.mjd_last_error.argtypes = []
        L.mjd_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def mjd_last_error() -> str:
    return lib().mjd_last_error().decode()


def _check(rc: int):
    if rc != MJD_OK:
        raise MjdError(rc, mjd_last_error())


def make_frame(frame) -> mjd_frame:
    """dict {width, height, h, v, qsel} (or an mjd_frame) -> mjd_frame."""
    if isinstance(frame, mjd_frame):
        return frame
    f = mjd_frame()
    f.width = int(frame["width"])
    f.height = int(frame["height"])
    for c in range(3):
        f.h[c] = int(frame["h"][c])
        f.v[c] = int(frame["v"][c])
        f.qsel[c] = int(frame.get("qsel", (0, 1, 1))[c])
    f.reserved = 0
    return f


def _ptr(x) -> int:
    """Address of a torch tensor, a numpy array or a raw integer address."""
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    return int(x.ctypes.data)


def _stream(s) -> int:
    if s is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


def mjd_geometry_of(frame) -> dict:
    g = mjd_geometry()
    _check(lib().mjd_geometry_of(ctypes.byref(make_frame(frame)), ctypes.byref(g)))
    return {"mcu_w": g.mcu_w, "mcu_h": g.mcu_h, "mcus_x": g.mcus_x, "mcus_y": g.mcus_y,
            "blocks_per_mcu": g.blocks_per_mcu, "comp_w": list(g.comp_w), "comp_h": list(g.comp_h),
            "n_blocks": g.n_blocks}


class Context:
    """Owns an mjd_ctx*; destroyed on close() or garbage collection."""

    def __init__(self, device: int = 0):
        p = ctypes.c_void_p()
        _check(lib().mjd_ctx_create(ctypes.byref(p), int(device)))
        self.handle = p
        self.device = device

    def close(self):
        if self.handle:
            lib().mjd_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mjd_ctx_create(device: int = 0) -> Context:
    return Context(device)


def mjd_ctx_destroy(ctx: Context):
    ctx.close()


def mjd_ctx_set_tuning(ctx: Context, seg_subtiles: int = 0, workgroups: int = 0, shape: int = 0):
    t = mjd_tuning(int(seg_subtiles), int(workgroups), int(shape))
    _check(lib().mjd_ctx_set_tuning(ctx.handle, ctypes.byref(t)))


def mjd_ctx_get_tuning(ctx: Context) -> dict:
    t = mjd_tuning()
    _check(lib().mjd_ctx_get_tuning(ctx.handle, ctypes.byref(t)))
    return {"seg_subtiles": t.seg_subtiles, "workgroups": t.workgroups, "shape": t.shape}


def mjd_shape_count(h: int, v: int, upsample: int) -> int:
    n = ctypes.c_uint32()
    _check(lib().mjd_shape_count(int(h), int(v), int(upsample), ctypes.byref(n)))
    return n.value


def mjd_shape_info(ctx: Context, h: int, v: int, upsample: int, index: int) -> dict:
    s = mjd_shape()
    _check(lib().mjd_shape_info(ctx.handle, int(h), int(v), int(upsample), int(index), ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in mjd_shape._fields_}


def mjd_decode(ctx: Context, frame, coef, qt, upsample: int, rgb, pitch: int,
               mcu_row0: int, mcu_row1: int, stream=None):
    _check(lib().mjd_decode(ctx.handle, ctypes.byref(make_frame(frame)), _ptr(coef), _ptr(qt),
                            int(upsample), _ptr(rgb), int(pitch), int(mcu_row0), int(mcu_row1),
                            _stream(stream)))


def mjd_decode_host(frame, coef, qt, upsample: int, rgb, pitch: int, row0: int, row1: int, n_threads: int = 1):
    """The decode on host cores (host arrays or pinned tensors)."""
    f = make_frame(frame)
    _check(lib().mjd_decode_host(ctypes.byref(f), _ptr(coef), _ptr(qt), int(upsample), _ptr(rgb), int(pitch),
                                 int(row0), int(row1), int(n_threads)))


def mjd_copy(ctx: Context, dst, src, nbytes: int, stream=None):
    _check(lib().mjd_copy(ctx.handle, _ptr(dst), _ptr(src), int(nbytes), _stream(stream)))


def _job_array(jobs):
    arr = (mjd_job * len(jobs))()
    for i, (frame, coef, qt, rgb, pitch) in enumerate(jobs):
        arr[i].frame = make_frame(frame)
        arr[i].d_coef = _ptr(coef)
        arr[i].d_qt = _ptr(qt)
        arr[i].d_rgb = _ptr(rgb)
        arr[i].pitch = int(pitch)
    return arr


class Batch:
    """Owns an mjd_batch*: a planned set of images decoded by one persistent launch."""

    def __init__(self, ctx: Context, jobs, upsample: int):
        arr = _job_array(jobs)
        p = ctypes.c_void_p()
        _check(lib().mjd_batch_create(ctx.handle, arr, len(jobs), int(upsample), ctypes.byref(p)))
        self.handle = p
        self._keep = jobs  # the device buffers must outlive the batch

    def info(self) -> dict:
        seg, wg, px = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
        _check(lib().mjd_batch_info(self.handle, ctypes.byref(seg), ctypes.byref(wg), ctypes.byref(px)))
        return {"segments": seg.value, "workgroups": wg.value, "pixels": px.value}

    def launch(self, use_graph: bool = False, stream=None):
        _check(lib().mjd_batch_launch(self.handle, int(bool(use_graph)), _stream(stream)))

    def close(self):
        if self.handle:
            lib().mjd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mjd_batch_create(ctx: Context, jobs, upsample: int) -> Batch:
    """jobs: sequence of (frame, coef, qt, rgb, pitch) with device tensors or addresses."""
    return Batch(ctx, jobs, upsample)


def mjd_batch_launch(batch: Batch, use_graph: bool = False, stream=None):
    batch.launch(use_graph, stream)


def mjd_batch_destroy(batch: Batch):
    batch.close()


def mjd_decode_batch_noalloc(ctx: Context, jobs, upsample: int, stream=None):
    """The batch decode of mjd_batch_create + launch, with no device allocation
    (the tables go into the library's fixed per-GPU array).  jobs: sequence of
    (frame, coef, qt, rgb, pitch); the buffers must outlive the kernel."""
    arr = _job_array(jobs)
    _check(lib().mjd_decode_batch_noalloc(ctx.handle, arr, len(jobs), int(upsample), _stream(stream)))


# ---- host side: bitstreams -> coefficients -------------------------------------------

def _bytes_view(jpg):
    import numpy as np
    a = np.frombuffer(jpg, dtype=np.uint8) if isinstance(jpg, (bytes, bytearray, memoryview)) else jpg
    return a, int(a.size)


def mjd_parse(jpg):
    """-> (mjd_scan, qt numpy uint16[4, 64])."""
    import numpy as np
    a, n = _bytes_view(jpg)
    scan = mjd_scan()
    qt = np.zeros((4, 64), dtype=np.uint16)
    _check(lib().mjd_parse(_ptr(a), n, ctypes.byref(scan), _ptr(qt)))
    return scan, qt


def mjd_restart_index(jpg, scan: mjd_scan):
    """-> numpy uint64[n_intervals + 1]."""
    import numpy as np
    a, n = _bytes_view(jpg)
    off = np.zeros(scan.n_intervals + 1, dtype=np.uint64)
    _check(lib().mjd_restart_index(_ptr(a), n, ctypes.byref(scan), _ptr(off)))
    return off


def mjd_entropy_decode(jpg, scan: mjd_scan, offsets, coef, row0: int, row1: int, n_threads: int = 1):
    """Decode MCU rows [row0, row1) into `coef` (host array or pinned tensor of n_blocks*64 int16)."""
    a, n = _bytes_view(jpg)
    _check(lib().mjd_entropy_decode(_ptr(a), n, ctypes.byref(scan), _ptr(offsets), _ptr(coef),
                                    int(row0), int(row1), int(n_threads)))


class EntropyBatch:
    """Owns an mjd_entropy_batch*: Huffman decoding of many scans on the GPU,
    one lane per restart interval."""

    def __init__(self, ctx: Context, jobs):
        """jobs: sequence of (scan, offsets, d_jpg, length, d_coef): the mjd_scan
        and restart index from mjd_parse / mjd_restart_index, the stream in
        device memory (tensor or address) with its byte length, and the
        device coefficient buffer of n_blocks*64 int16."""
        arr = (mjd_entropy_job * len(jobs))()
        for i, (scan, off, jpg, n, coef) in enumerate(jobs):
            arr[i].scan = ctypes.pointer(scan)
            arr[i].h_offsets = _ptr(off)
            arr[i].d_jpg = _ptr(jpg)
            arr[i].len = int(n)
            arr[i].d_coef = _ptr(coef)
        p = ctypes.c_void_p()
        _check(lib().mjd_entropy_batch_create(ctx.handle, arr, len(jobs), ctypes.byref(p)))
        self.handle = p
        self._keep = jobs  # the device buffers must outlive the batch

    def info(self) -> dict:
        iv, wg, nb = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
        _check(lib().mjd_entropy_batch_info(self.handle, ctypes.byref(iv), ctypes.byref(wg), ctypes.byref(nb)))
        return {"intervals": iv.value, "workgroups": wg.value, "bytes": nb.value}

    def launch(self, stream=None):
        _check(lib().mjd_entropy_batch_launch(self.handle, _stream(stream)))

    def status(self) -> int:
        """Synchronise; raise MjdError (MJD_ECORRUPT) for corrupt data, else -1."""
        bad = ctypes.c_int64(-1)
        rc = lib().mjd_entropy_batch_status(self.handle, ctypes.byref(bad))
        if rc != MJD_OK:
            err = MjdError(rc, mjd_last_error())
            err.bad_job = bad.value
            raise err
        return bad.value

    def close(self):
        if self.handle:
            lib().mjd_entropy_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mjd_entropy_batch_create(ctx: Context, jobs) -> EntropyBatch:
    return EntropyBatch(ctx, jobs)


def mjd_entropy_batch_launch(batch: EntropyBatch, stream=None):
    batch.launch(stream)


def mjd_entropy_batch_status(batch: EntropyBatch) -> int:
    return batch.status()


def mjd_entropy_batch_info(batch: EntropyBatch) -> dict:
    return batch.info()


def mjd_entropy_batch_destroy(batch: EntropyBatch):
    batch.close()


# ---- performance model (paper Sec. 5.1) ---------------------------------------------

def _dbl(v):
    import numpy as np
    a = np.ascontiguousarray(v, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def mjd_poly1_fit(x, y, max_degree: int = 7):
    """-> (mjd_poly1, AIC) of the least-AIC least-squares fit."""
    xa, xp = _dbl(x)
    ya, yp = _dbl(y)
    if len(xa) != len(ya):
        raise ValueError("x and y differ in length")
    out, aic = mjd_poly1(), ctypes.c_double()
    _check(lib().mjd_poly1_fit(xp, yp, len(ya), int(max_degree), ctypes.byref(out), ctypes.byref(aic)))
    return out, aic.value


def mjd_poly2_fit(a, b, y, max_degree: int = 7):
    """-> (mjd_poly2, AIC) of the least-AIC least-squares fit in (a, b)."""
    aa, ap = _dbl(a)
    ba, bp = _dbl(b)
    ya, yp = _dbl(y)
    if not len(aa) == len(ba) == len(ya):
        raise ValueError("a, b and y differ in length")
    out, aic = mjd_poly2(), ctypes.c_double()
    _check(lib().mjd_poly2_fit(ap, bp, yp, len(ya), int(max_degree), ctypes.byref(out), ctypes.byref(aic)))
    return out, aic.value


def mjd_poly1_eval(p: mjd_poly1, x: float) -> float:
    return lib().mjd_poly1_eval(ctypes.byref(p), float(x))


def mjd_poly2_eval(p: mjd_poly2, a: float, b: float) -> float:
    return lib().mjd_poly2_eval(ctypes.byref(p), float(a), float(b))


def mjd_model_predict(model: mjd_model, width: int, height: int, file_bytes: int) -> dict:
    out = mjd_prediction()
    _check(lib().mjd_model_predict(ctypes.byref(model), int(width), int(height), int(file_bytes),
                                   ctypes.byref(out)))
    return {k: getattr(out, k) for k, _ in mjd_prediction._fields_}


def mjd_partition_rows(model: mjd_model, scheme: int, width: int, height: int, mcu_h: int, file_bytes: int,
                       huff_threads: float = 1.0, chunk_rows: int = 0) -> dict:
    out = mjd_partition()
    _check(lib().mjd_partition_rows(ctypes.byref(model), int(scheme), int(width), int(height), int(mcu_h),
                                    int(file_bytes), float(huff_threads), int(chunk_rows), ctypes.byref(out)))
    return {k: getattr(out, k) for k, _ in mjd_partition._fields_}


def mjd_repartition_rows(model: mjd_model, width: int, height: int, rows_left: int, mcu_h: int, file_bytes: int,
                         huff_threads: float, huff_rows_left: int, huff_done_s: float, gpu_busy_s: float) -> dict:
    out = mjd_partition()
    _check(lib().mjd_repartition_rows(ctypes.byref(model), int(width), int(height), int(rows_left), int(mcu_h),
                                      int(file_bytes), float(huff_threads), int(huff_rows_left), float(huff_done_s),
                                      float(gpu_busy_s), ctypes.byref(out)))
    return {k: getattr(out, k) for k, _ in mjd_partition._fields_}


def make_variant(frame, ncomp: int = 3, idct: str = "islow", mode: str = "fancy", scale: int = 1) -> mjd_variant:
    """frame dict (as for make_frame; grayscale may give width, height and
    qsel only) -> mjd_variant."""
    f = dict(frame)
    f.setdefault("h", (1, 1, 1))
    f.setdefault("v", (1, 1, 1))
    q = tuple(f.get("qsel", (0, 0, 0))) + (0, 0, 0)
    f["qsel"] = q[:3]
    return mjd_variant(frame=make_frame(f), ncomp=int(ncomp), idct=IDCT[idct],
                       upsample=MJD_UPSAMPLE_FANCY if mode == "fancy" else MJD_UPSAMPLE_SIMPLE, scale=int(scale))


def mjd_variant_geometry(variant: mjd_variant) -> tuple:
    """-> (geometry dict, workspace bytes)."""
    g = mjd_geometry()
    wb = ctypes.c_uint64()
    _check(lib().mjd_variant_geometry(ctypes.byref(variant), ctypes.byref(g), ctypes.byref(wb)))
    return ({"mcu_w": g.mcu_w, "mcu_h": g.mcu_h, "mcus_x": g.mcus_x, "mcus_y": g.mcus_y,
             "blocks_per_mcu": g.blocks_per_mcu, "comp_w": list(g.comp_w), "comp_h": list(g.comp_h),
             "n_blocks": g.n_blocks}, wb.value)


def mjd_decode_variant(ctx: Context, variant: mjd_variant, coef, qt, out, pitch: int, work, work_bytes: int,
                       stream=None):
    _check(lib().mjd_decode_variant(ctx.handle, ctypes.byref(variant), _ptr(coef), _ptr(qt), _ptr(out),
                                    int(pitch), _ptr(work), int(work_bytes), _stream(stream)))


class Hetero:
    """Owns an mjd_hetero*: CPU-GPU partitioned decode of one image at a time."""

    def __init__(self, ctx: Context, max_blocks: int, max_pixels: int, n_threads: int = 16):
        p = ctypes.c_void_p()
        _check(lib().mjd_hetero_create(ctx.handle, int(max_blocks), int(max_pixels), int(n_threads),
                                       ctypes.byref(p)))
        self.handle = p

    def decode(self, jpg, rgb, pitch: int, cpu_rows: int, scheme: int = MJD_PART_SPS,
               upsample: int = MJD_UPSAMPLE_FANCY, chunk_mcu_rows: int = 0, model: mjd_model | None = None,
               huff_threads: float = 1.0) -> dict:
        a, n = _bytes_view(jpg)
        plan = mjd_hetero_plan(scheme=int(scheme), cpu_rows=int(cpu_rows), chunk_mcu_rows=int(chunk_mcu_rows),
                               model=ctypes.cast(ctypes.pointer(model), ctypes.c_void_p) if model is not None else None,
                               huff_threads=float(huff_threads))
        t = mjd_hetero_times()
        _check(lib().mjd_hetero_decode(self.handle, _ptr(a), n, int(upsample), ctypes.byref(plan), _ptr(rgb),
                                       int(pitch), ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in mjd_hetero_times._fields_}

    def close(self):
        if self.handle:
            lib().mjd_hetero_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def scan_frame(scan: mjd_scan) -> dict:
    """The frame of a parsed scan; grayscale frames carry "ncomp": 1."""
    f = scan.frame
    d = {"width": f.width, "height": f.height, "h": tuple(f.h), "v": tuple(f.v), "qsel": tuple(f.qsel)}
    if scan.ncomp == 1:
        d["ncomp"] = 1
    return d


class Pipeline:
    """Owns an mjd_pipeline*: host entropy workers + pinned slots + three streams."""

    def __init__(self, ctx: Context, n_threads: int, max_blocks: int, max_pixels: int, upsample: int = 1,
                 n_slots: int = 3, band_mcu_rows: int = 0):
        cfg = mjd_pipeline_config(n_threads=int(n_threads), n_slots=int(n_slots),
                                  band_mcu_rows=int(band_mcu_rows), upsample=int(upsample),
                                  max_blocks=int(max_blocks), max_pixels=int(max_pixels))
        p = ctypes.c_void_p()
        _check(lib().mjd_pipeline_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(p)))
        self.handle = p
        self.ctx = ctx

    def run(self, jpgs, outs, pitches=None, entropy_only: bool = False) -> dict:
        """jpgs: sequence of bytes / uint8 arrays; outs: host buffers (numpy or
        pinned tensors) of H*pitch bytes each.  Returns the run's statistics."""
        n = len(jpgs)
        views = [_bytes_view(j) for j in jpgs]
        ptrs = (ctypes.c_void_p * n)(*[_ptr(a) for a, _ in views])
        lens = (ctypes.c_size_t * n)(*[ln for _, ln in views])
        outp = (ctypes.c_void_p * n)(*[_ptr(o) for o in outs])
        if pitches is None:
            pitches = [int(o.shape[1]) * int(o.shape[2]) for o in outs]
        pit = (ctypes.c_size_t * n)(*[int(x) for x in pitches])
        st = mjd_pipeline_stats()
        flags = MJD_PIPELINE_ENTROPY_ONLY if entropy_only else 0
        _check(lib().mjd_pipeline_run(self.handle, n, ptrs, lens, outp, pit, flags, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in mjd_pipeline_stats._fields_}

    def close(self):
        if self.handle:
            lib().mjd_pipeline_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Owns an mjd_server*: the continuous-batching (or synchronous) request loop."""

    def __init__(self, ctx: Context, budget_bytes: int, upsample: int = 1, mode: int = MJD_SERVE_CONTINUOUS,
                 max_batch: int = 256, max_inflight: int = 2, model=None, max_batch_s: float = 0.0):
        """model (an mjd_model) and max_batch_s cap each batch's predicted GPU time."""
        cfg = mjd_server_config(budget_bytes=int(budget_bytes), upsample=int(upsample), mode=int(mode),
                                max_batch=int(max_batch), max_inflight=int(max_inflight),
                                model=ctypes.addressof(model) if model is not None else None,
                                max_batch_s=float(max_batch_s))
        p = ctypes.c_void_p()
        _check(lib().mjd_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(p)))
        self.handle = p
        self._keep = {}

    def now_ns(self) -> int:
        return int(lib().mjd_server_now_ns(self.handle))

    def submit(self, frame, coef, qt, rgb, pitch: int, arrival_ns: int = 0) -> int:
        """coef/qt: host buffers (pinned tensors or numpy arrays); rgb: a host
        buffer, or a CUDA tensor on the server's device (the kernel writes it,
        nothing is copied back).  All stay alive until done."""
        on_device = bool(getattr(rgb, "is_cuda", False))
        r = mjd_request(frame=make_frame(frame), h_coef=_ptr(coef), h_qt=_ptr(qt),
                        h_rgb=None if on_device else _ptr(rgb), d_rgb=_ptr(rgb) if on_device else None,
                        pitch=int(pitch), arrival_ns=int(arrival_ns))
        rid = ctypes.c_uint64()
        _check(lib().mjd_server_submit(self.handle, ctypes.byref(r), ctypes.byref(rid)))
        self._keep[rid.value] = (coef, qt, rgb)
        return rid.value

    def wait(self, rid: int) -> dict:
        t = mjd_request_times()
        rc = lib().mjd_server_wait(self.handle, int(rid), ctypes.byref(t))
        self._keep.pop(rid, None)
        out = {k: getattr(t, k) for k, _ in mjd_request_times._fields_}
        if rc != MJD_OK:
            raise MjdError(rc, mjd_last_error())
        return out

    def drain(self):
        _check(lib().mjd_server_drain(self.handle))

    def close(self):
        if self.handle:
            lib().mjd_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
