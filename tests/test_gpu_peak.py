"""The attainable-peak probes that the roofline fractions are also quoted
against: the matrix-core loop returns its exact sum (every operand equals
`one`, so each lane ends with 128 * iters * one^2), the streaming read returns
the XOR of every word it read, the streaming copy copies (ragged tails
included), and bad arguments are rejected on the host."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("bits", [64, 32])
def test_peak_mfma_exact_sum(bits):
    import torch
    from paper_2608_27863_amd import hdg
    dt = torch.float64 if bits == 64 else torch.float32
    for n_wg, iters, one in ((3, 5, 0.5), (17, 1000, 1.0)):
        print(f"[peak] FP{bits} n_wg={n_wg} iters={iters} one={one}", flush=True)
        sink = torch.full((n_wg * 256,), -1.0, dtype=dt, device="cuda")
        hdg.hdg_peak_mfma(bits, n_wg, iters, one, sink)
        torch.cuda.synchronize()
        assert bool((sink == 128.0 * iters * one * one).all().item())


def test_peak_copy_copies():
    import torch
    from paper_2608_27863_amd import hdg
    g = torch.Generator(device="cuda").manual_seed(3)
    for nbytes in (16, 16 * 1001, 16 * (4096 * 1024 * 2 + 4096 * 3 + 77)):  # several chunks per workgroup, a ragged last chunk
        print(f"[peak] copy {nbytes} bytes", flush=True)
        src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
        dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
        hdg.hdg_peak_copy(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(dst[:nbytes], src) and not dst[nbytes:].any().item()


def test_peak_read_xor():
    import numpy as np
    import torch
    from paper_2608_27863_amd import hdg
    g = torch.Generator(device="cuda").manual_seed(5)
    for nbytes in (16, 16 * 1001, 16 * (4096 * 1024 * 3 + 4096 * 5 + 129)):  # several chunks per workgroup, a ragged last chunk
        print(f"[peak] read {nbytes} bytes", flush=True)
        src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
        sink = torch.zeros(1, dtype=torch.int32, device="cuda")
        hdg.hdg_peak_read(src, sink)
        torch.cuda.synchronize()
        words = src.cpu().numpy().view(np.uint32)
        assert int(sink.cpu().numpy().view(np.uint32)[0]) == int(np.bitwise_xor.reduce(words))


def test_peak_argument_errors():
    import torch
    from paper_2608_27863_amd import hdg
    L = hdg.load_library()
    INVALID = -1  # HDG_ERR_INVALID_ARGUMENT
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    p = buf.data_ptr()
    vp = ctypes.c_void_p
    # every call below is rejected before any launch
    assert L.hdg_peak_mfma(16, 1, 1, 1.0, vp(p), None) == INVALID
    assert L.hdg_peak_mfma(64, 0, 1, 1.0, vp(p), None) == INVALID
    assert L.hdg_peak_mfma(64, 1, 0, 1.0, vp(p), None) == INVALID
    assert L.hdg_peak_mfma(64, 1, 1, 1.0, None, None) == INVALID
    assert L.hdg_peak_read(vp(p), 24, vp(p + 2048), None) == INVALID      # not a multiple of 16
    assert L.hdg_peak_read(vp(p + 8), 32, vp(p + 2048), None) == INVALID  # misaligned
    assert L.hdg_peak_read(vp(p), 32, None, None) == INVALID
    assert L.hdg_peak_copy(vp(p), vp(p + 2048), 24, None) == INVALID     # not a multiple of 16
    assert L.hdg_peak_copy(vp(p + 8), vp(p + 2048), 32, None) == INVALID  # misaligned
    assert L.hdg_peak_copy(vp(p), vp(p + 1024), 2048, None) == INVALID    # overlapping
    assert L.hdg_peak_copy(vp(p), vp(p + 2048), 0, None) == INVALID
    assert L.hdg_peak_copy(None, vp(p), 16, None) == INVALID
    torch.cuda.synchronize()
    assert not buf.any().item()
