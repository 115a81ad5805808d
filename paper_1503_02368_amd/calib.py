"""Plain device copy of a known size, used to calibrate rocprofv3 memory
counters: run it under ``rocprofv3 --pmc FETCH_SIZE`` (then WRITE_SIZE) and
divide the known bytes by what the counter reports per dispatch.

    python -m paper_1503_02368_amd.calib [MiB]

``probe_gbs(ctx)`` times the library's hand-written streaming-read kernel
over a buffer larger than the last-level cache: the read bandwidth a plain
read-only kernel reaches on this GPU, the achievable ceiling beside the
8 TB/s nominal peak.
"""
import sys


def probe_gbs(ctx, mib: int = 4096, reps: int = 10, blocks=(4, 8, 16, 32)) -> dict:
    """GB/s of the library's streaming-read kernel (eh_stream_read: 128-bit
    loads over a grid-stride loop, every byte read once) over `mib` MiB, far
    larger than the 256 MB last-level cache, timed with HIP events on the
    context's stream over `reps` launches after a warm-up, for each count of
    blocks per compute unit in `blocks`.  read = the best of them."""
    import torch
    nbytes = mib * (1 << 20)
    buf = torch.zeros(nbytes // 8, dtype=torch.int64, device="cuda")
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = ctx.stream
    s.wait_stream(torch.cuda.current_stream())
    by_blocks = {}
    for b in blocks:
        ctx.stream_read_async(buf, sink, b)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            ctx.stream_read_async(buf, sink, b)
        e1.record(s)
        torch.cuda.synchronize()
        by_blocks[str(b)] = nbytes / (e0.elapsed_time(e1) / reps / 1e3) / 1e9
    del buf, sink
    torch.cuda.empty_cache()
    return {"read": max(by_blocks.values()), "read_by_blocks_per_cu": by_blocks,
            "kernel": "k_stream_read", "mib": mib}


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
