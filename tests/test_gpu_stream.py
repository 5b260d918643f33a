"""The bandwidth probes behind the roofline's measured denominator: STREAM's
triad and the chunked read pass, element by element against host arithmetic,
over empty, ragged and multi-chunk lengths."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 5, 2047, 2048, 2049, 3 * 4096 + 7, 1 << 20]


@pytest.mark.parametrize("n", SIZES)
def test_triad_matches_host(n):
    import torch

    from paper_2004_09389_amd.hdg import stream_triad
    print(f"[stream] triad n={n}", flush=True)
    rng = np.random.default_rng(n + 1)
    b, c = rng.standard_normal(n), rng.standard_normal(n)
    a = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    stream_triad(torch.from_numpy(b).cuda(), torch.from_numpy(c).cuda(), -2.5, a)
    got = a.cpu().numpy()
    ref = b + (-2.5) * c
    # the kernel may contract to one fused multiply-add: at most one rounding apart
    assert np.all(np.abs(got - ref) <= 2.0 ** -52 * (np.abs(b) + 2.5 * np.abs(c)))


@pytest.mark.parametrize("n", SIZES)
def test_read_partials_are_the_chunk_sums(n):
    import torch

    from paper_2004_09389_amd.hdg import stream_read, stream_read_blocks
    print(f"[stream] read n={n}", flush=True)
    x = np.random.default_rng(n + 2).standard_normal(n)
    nb = stream_read_blocks(n)
    assert nb == -(-n // 2048)
    partial = torch.full((nb + 3,), 7.0, dtype=torch.float64, device="cuda")
    stream_read(torch.from_numpy(x).cuda(), partial)
    got = partial.cpu().numpy()
    for k in range(nb):
        chunk = x[2048 * k:2048 * (k + 1)]
        assert abs(got[k] - math.fsum(chunk)) <= 1e-14 * np.abs(chunk).sum()
    assert np.all(got[nb:] == 7.0)  # nothing written past the chunks


def test_probes_reject_misaligned_and_short_buffers():
    import torch

    from paper_2004_09389_amd.hdg import HdgError, stream_read, stream_triad
    x = torch.zeros(4097, dtype=torch.float64, device="cuda")
    with pytest.raises(HdgError):
        stream_triad(x[1:], x[1:].clone(), 1.0, torch.zeros(4096, dtype=torch.float64, device="cuda"))
    with pytest.raises(HdgError):
        stream_read(x, torch.zeros(2, dtype=torch.float64, device="cuda"))
