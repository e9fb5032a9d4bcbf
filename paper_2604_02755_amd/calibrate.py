"""HBM traffic calibration: a plain device copy of known size.

Run under ``rocprofv3 --pmc FETCH_SIZE`` (then ``WRITE_SIZE``) next to the
benchmark: the ratio of what the counters report for this copy (1 GiB read,
1 GiB written per dispatch) to the true bytes scales the counters taken on the
solver's kernels.  Also prints the achieved copy bandwidth.
"""
from __future__ import annotations

import sys
import time


def main(n_bytes: int = 1 << 30, reps: int = 5) -> None:
    import torch
    n = n_bytes // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.mul(x, 1.0, out=y)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(f"copy of {n_bytes} B: {2 * n_bytes / dt / 1e9:.1f} GB/s (read + write), {reps + 1} dispatches",
          flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else (1 << 30))
