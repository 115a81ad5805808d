"""Plain device copy of a known size, used to calibrate rocprofv3 memory
counters: run it under ``rocprofv3 --pmc FETCH_SIZE`` (then WRITE_SIZE) and
divide the known bytes by what the counter reports per dispatch.

    python -m paper_1503_02368_amd.calib [MiB]

``probe_gbs()`` measures the bandwidth a plain streaming read and a copy
reach on this GPU (the achievable ceiling beside the 8 TB/s nominal peak).
"""
import sys


def probe_gbs(mib: int = 4096, reps: int = 10) -> dict:
    """GB/s of a streaming read and of a copy (read + write) over `mib` MiB,
    timed with HIP events over `reps` repetitions after a warm-up.  The read
    figure is the best of three plain reductions over float32 data (sum, max
    and a norm), each of which reads every byte once."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)

    def gbs(fn, factor):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return factor * n * 4 / (e0.elapsed_time(e1) / reps / 1e3) / 1e9

    reads = {"sum": gbs(lambda: a.sum(), 1), "max": gbs(lambda: a.amax(), 1),
             "norm": gbs(lambda: torch.linalg.vector_norm(a, 1), 1)}
    out = {"read": max(reads.values()), "read_by_op": reads, "copy": gbs(lambda: b.copy_(a), 2)}
    del a, b
    torch.cuda.empty_cache()
    return out


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
