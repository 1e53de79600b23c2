"""Seeded synthetic inputs for the JPEG back-half decoder.

Shared by the tests, the benchmark and the oracle's checks.  This package
holds only input generation (pixel content, the encoder side of JPEG, quant
tables, bitstream writing); it contains none of the decoder's arithmetic.
"""
from .encode import SAMPLINGS, encode_rgb, make_frame, mcu_grid  # noqa: F401
from .tables import quant_tables  # noqa: F401
