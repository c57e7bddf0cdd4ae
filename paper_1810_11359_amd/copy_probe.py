"""Plain device-to-device copy of a known size, used to calibrate the HBM
traffic counters (FETCH_SIZE / WRITE_SIZE) that rocprofv3 reports for the ISM
kernels: run it under the same --pmc pass and divide."""
import sys

import torch


def main(mib: int = 256) -> None:
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x 3", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 256)
