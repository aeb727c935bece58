"""Plain device-to-device copies of a known size, for calibrating hardware
byte counters (run it under a counter-collecting profiler and divide the
known bytes by what the counter reports for these dispatches).

    python -m paper_2404_17542_amd.copy_calibration --mib 1024 --reps 5
"""
from __future__ import annotations

import argparse

import torch


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024, help="bytes copied per dispatch, in MiB")
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args(argv)
    n = a.mib * (1 << 20) // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    assert torch.equal(dst[:: 1 << 16], src[:: 1 << 16])
    print(f"copied {a.mib} MiB x {a.reps} (read {a.mib} MiB and write {a.mib} MiB per dispatch)", flush=True)


if __name__ == "__main__":
    main()
