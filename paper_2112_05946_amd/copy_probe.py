"""Device copy of a known size with the library's streaming copy kernel
(fr_sg_copy): the run whose FETCH_SIZE / WRITE_SIZE readings calibrate the HBM
byte counters against which the stage kernels' traffic is scaled."""

import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import torch  # noqa: E402

from paper_2112_05946_amd.binding import device_copy  # noqa: E402

NBYTES = 1 << 30  # 1 GiB read + 1 GiB written per copy


def main():
    torch.cuda.set_device(0)
    a = torch.ones(NBYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        device_copy(a, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    print("copied %d bytes x 3 with k_copy" % NBYTES, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
