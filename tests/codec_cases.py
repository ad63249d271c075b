"""Shared inputs of the row-codec tests (the oracle twin on the CPU and the GPU kernels)."""
import numpy as np


def rows_fixture():
    """Rows of 700 points (not a multiple of 64, longer than 512) with magnitudes spread over many
    decades per row, plus an all-zero row, a row whose maximum is an FP32 subnormal and exact ties."""
    rng = np.random.default_rng(17)
    nz, ny, nx = 3, 5, 700
    f = (rng.standard_normal((nz, ny, nx)) * 10.0 ** rng.uniform(-4, 1, (nz, ny, nx))
         * 10.0 ** rng.uniform(-3, 3, (nz, ny, 1))).astype(np.float32)
    f[0, 1] = 0.0
    f[1, 2] = np.float32(1e-40) * rng.uniform(-1, 1, nx).astype(np.float32)
    f[2, 3, :4] = np.array([1 + 2 ** -11, 1 + 3 * 2 ** -11, -(1 + 2 ** -8), 0.5 + 2 ** -9], np.float32)
    f[2, 3, 4] = 2.0
    return f
