"""The streaming-read probe reads every byte once: its fold (XOR of every
32-bit word) equals numpy's over the same buffer, for sizes that leave a
ragged tail past the four-loads-per-lane loop, and bad sizes are refused."""
import numpy as np
import pytest

from paper_1503_02368_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("words,blocks", [(4, 0), (4 * 1000 + 8, 1), (1 << 20, 8),
                                          ((3 << 20) + 44, 64)])
def test_stream_read_fold(eh, words, blocks):
    import torch
    ctx = eh.Context(0)
    try:
        host = inputs.rand_u64(inputs.stream_key(77, words), 0, words // 2).view(np.uint32)
        buf = torch.from_numpy(host.view(np.int32)).cuda()
        sink = torch.zeros(1, dtype=torch.int64, device="cuda")
        ctx.stream.wait_stream(torch.cuda.current_stream())
        ctx.stream_read_async(buf, sink, blocks)
        torch.cuda.synchronize()
        want = np.bitwise_xor.reduce(host)
        assert int(sink.cpu().numpy().view(np.uint64)[0]) == int(want)
        # a second pass folds the same words again: XOR returns to zero
        ctx.stream_read_async(buf, sink, blocks)
        torch.cuda.synchronize()
        assert int(sink.cpu().numpy().view(np.uint64)[0]) == 0
        with pytest.raises(eh.EHError) as e:
            ctx.stream_read_async(buf[:3], sink, blocks)
        assert e.value.status == eh.EH_EINVAL
        with pytest.raises(eh.EHError) as e:
            ctx.stream_read_async(buf, sink, 65)
        assert e.value.status == eh.EH_EINVAL
    finally:
        ctx.close()
