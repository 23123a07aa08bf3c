"""The bandwidth probe's kernels do exactly what their traffic assumes: a
copy reproduces the source bit for bit, the read pass's XOR checksums of
8 KiB blocks equal the host's, the fill writes the value everywhere (ragged
sizes included)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096 * 16 + 48, (64 << 20) + 16 * 7])
def test_probe_kernels(nbytes):
    import torch
    import paper_2110_13055_amd as P
    print(f"probe bytes={nbytes}", flush=True)
    g = torch.Generator().manual_seed(nbytes)
    host = torch.randint(0, 2 ** 31 - 1, (nbytes // 4,), dtype=torch.int32, generator=g)
    src = host.cuda()
    dst = torch.zeros_like(src)
    P.bandwidth_probe(P.PROBE_COPY, dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst.cpu(), host)
    nblk = -(-nbytes // 8192)
    chk = torch.full((4 * nblk,), 7, dtype=torch.int32, device="cuda")
    P.bandwidth_probe(P.PROBE_READ, chk, src)
    torch.cuda.synchronize()
    words = host.numpy().view(np.uint32).reshape(-1, 4)
    pad = np.zeros((nblk * 512, 4), np.uint32)
    pad[:words.shape[0]] = words
    ref = np.bitwise_xor.reduce(pad.reshape(nblk, 512, 4), axis=1)
    assert np.array_equal(chk.cpu().numpy().view(np.uint32).reshape(nblk, 4), ref)
    P.bandwidth_probe(P.PROBE_FILL, dst, None, value=0x12345678)
    torch.cuda.synchronize()
    assert bool((dst == 0x12345678).all())


def test_probe_rejects_bad_arguments():
    import torch
    import paper_2110_13055_amd as P
    a = torch.zeros(64, dtype=torch.int32, device="cuda")
    with pytest.raises(P.CdiError):
        P.bandwidth_probe(P.PROBE_COPY, a, a)             # overlapping
    with pytest.raises(P.CdiError):
        P.bandwidth_probe(P.PROBE_COPY, a[1:5], a[8:12])  # misaligned
    with pytest.raises(P.CdiError):
        P.bandwidth_probe(7, a, a)
