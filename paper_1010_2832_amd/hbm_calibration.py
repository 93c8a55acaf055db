"""Plain device copy of known size, for scaling rocprofv3 FETCH_SIZE /
WRITE_SIZE readings into bytes: y = x + 0 over N float32 values reads
exactly 4N bytes and writes 4N bytes of HBM (N*4 = 1 GiB by default, far
larger than every cache level).  Run it under rocprofv3 --pmc with
--kernel-include-regex matching the elementwise kernel and divide the known
bytes by the counter reading to get the scale factor."""
import argparse
import json

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    n = args.mib * 1024 * 1024 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(args.reps):
        torch.add(x, 0.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "reps": args.reps}))


if __name__ == "__main__":
    main()
