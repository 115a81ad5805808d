"""Plain device copy of a known size, used to calibrate rocprofv3 memory
counters: run it under ``rocprofv3 --pmc FETCH_SIZE`` (then WRITE_SIZE) and
divide the known bytes by what the counter reports per dispatch.

    python -m paper_1503_02368_amd.calib [MiB]
"""
import sys


def main():
    import torch
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    n = mib * (1 << 20) // 4
    a = torch.arange(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB three times ({3 * n * 4} bytes read, {3 * n * 4} written)")


if __name__ == "__main__":
    main()
