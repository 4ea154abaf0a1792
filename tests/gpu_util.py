"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
compare with the oracle."""
import numpy as np


def device():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_device(text: bytes):
    import torch
    a = np.frombuffer(text, dtype=np.uint8) if not isinstance(text, np.ndarray) else text
    t = torch.empty(max(a.size, 1), dtype=torch.uint8, device=device())
    if a.size:
        t[:a.size].copy_(torch.from_numpy(a.copy()))
    return t[:a.size]


class ParseResult(tuple):
    """A tuple (columns, accepted, count mod 2^64, count status[, trace]) that
    also carries the count modulo 2^61 - 1 as ``.countp``."""
    countp = 0


def gpu_parse(parser, text, chunk_bytes=0, count=True, force_l2=False, trace=False, flags=0):
    """(columns uint64 [n+1, W], accepted, count, count_status[, trace uint64 [2, c+1, W]]),
    with ``.countp`` the count modulo 2^61 - 1."""
    import torch
    t = to_device(text) if not hasattr(text, "device") else text
    res = parser.parse(t, chunk_bytes=chunk_bytes, count=count, force_l2=force_l2, trace=trace, flags=flags)
    torch.cuda.synchronize()
    cols = res[0].cpu().numpy().view(np.uint64)
    sc = res[1].cpu().numpy().view(np.uint64)
    out = (cols, bool(sc[0]), int(sc[1]), int(sc[2]))
    if trace:
        out = out + (res[2].cpu().numpy().view(np.uint64),)
    out = ParseResult(out)
    out.countp = int(sc[3])
    return out
