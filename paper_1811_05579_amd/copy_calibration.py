"""Plain device-to-device copy of a known size, run under rocprofv3 --pmc to
calibrate the FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch) that the
kernel profiles in profiles/ are scaled by: the copy reads and writes exactly
MIB MiB per launch."""
import sys

import torch

MIB = 256


def main():
    n = MIB * 2 ** 20 // 8
    x = torch.arange(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    assert bool((y[-4:] == x[-4:]).all())
    print(f"copied {MIB} MiB x 3 launches", flush=True)


if __name__ == "__main__":
    sys.exit(main())
