"""CPU oracle for the JPEG back half: dequantise -> islow IDCT -> chroma
upsampling -> YCbCr->RGB, plus a baseline Huffman JPEG reader.

TEST INFRASTRUCTURE ONLY.  This package is plain, slow, obviously-correct
numpy written from the paper's description of the decoder (Sec. 2, Sec. 4.1
Eqs. 1-2, Sec. 4.2 Algorithm 1, Sec. 4.3 Algorithm 2) and from T.81 where the
paper is silent.  It defines the bits every GPU result must match.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import it; the
product library never calls it and shares no code, tables or constants with
it.

Every function here is pinned by tests against something other than itself
(closed forms, FP64 transforms, brute force, the paper's Algorithm 1 and an
independent libjpeg-turbo build run as a black box).
"""
from .colour import ycc_to_rgb  # noqa: F401
from .decode import component_planes, decode, decode_rows  # noqa: F401
from .geometry import geometry  # noqa: F401
from .idct import dequantise, idct_blocks  # noqa: F401
from .jfif import JpegError, parse_and_decode  # noqa: F401
from .upsample import upsample  # noqa: F401
