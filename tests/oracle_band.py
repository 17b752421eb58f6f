"""One band of rows of the FP64 oracle's output on the 1080p workload frame.

Run as a child process by the full-frame parity test (several bands at once,
one thread each): the frame is regenerated from its seed, the oracle is
evaluated on rows [y0, y1) (with the 2r halo the block evaluation takes),
and the band is saved as a float64 .npy file.

    python tests/oracle_band.py Y0 Y1 OUT.npy
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import flr_ref as ref  # noqa: E402
from synth import make_config  # noqa: E402

# The regulariser the library receives: flr_params.eps is FP32, and at the
# few windows whose fits are nearly singular, rounding 1e-3 to FP32 alone
# moves the exact output by up to 1e-4 relative (the tolerance itself).
RADIUS, EPS = 8, float(np.float32(1e-3))


def main(argv) -> int:
    y0, y1, path = int(argv[1]), int(argv[2]), argv[3]
    fr = make_config(1)
    W = fr["noisy"].shape[-1]
    band = ref.flr_reference_block(fr["noisy"], fr["guides"], RADIUS, EPS, y0, y1, 0, W)
    np.save(path, np.asarray(band, dtype=np.float64))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
