"""Streaming-copy calibration: achievable device bandwidth and the scale
factor of the hardware byte counters.

Runs ``wl_stream_copy`` on a buffer of known size (default 1 GiB) several
times and prints the achieved read+write bandwidth.  Under
``rocprofv3 --pmc FETCH_SIZE`` (and, in a separate run, ``WRITE_SIZE``) each
copy dispatch reads and writes exactly ``--mib`` MiB, so counter / known
bytes gives the factor used to turn the stencil's counters into HBM bytes.

Usage: python -m paper_1712_01505_amd.calibrate [--mib 1024] [--reps 5]
"""
import argparse
import json
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    import torch

    from . import wilson as W

    n = a.mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    st = W._stream()
    W.wl_stream_copy(dst.data_ptr(), src.data_ptr(), n, st)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.reps):
        W.wl_stream_copy(dst.data_ptr(), src.data_ptr(), n, st)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / a.reps
    if not torch.equal(src[:: 1 << 20], dst[:: 1 << 20]):
        raise SystemExit("copy check failed")
    print(json.dumps({"kernel": "stream_copy_kernel", "bytes_read": n, "bytes_written": n, "dispatches": a.reps + 1,
                      "avg_us": round(ms * 1e3, 2), "GB/s_read_plus_write": round(2 * n / (ms * 1e-3) / 1e9, 1)}))
    sys.stdout.flush()


if __name__ == "__main__":
    main()
