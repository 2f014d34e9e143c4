"""Plain device copy of a known size, used to calibrate the HBM byte counters
(FETCH_SIZE / WRITE_SIZE) against which the stage kernels' traffic is scaled."""

import sys

import torch

NBYTES = 1 << 30  # 1 GiB read + 1 GiB written per copy


def main():
    torch.cuda.set_device(0)
    a = torch.ones(NBYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied %d bytes x 3" % NBYTES, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
