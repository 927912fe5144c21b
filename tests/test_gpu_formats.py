"""The GPU's number-format conversions against the oracle's, bit for bit:
FP32 -> BF16 rounding (both forms the kernels use) over every FP32 bit
pattern but NaN, and the per-row e4m3 weight quantiser of the FP8-weight
precision with rounding ties, subnormals, zero rows and saturation."""
import concurrent.futures as cf
import sys

import numpy as np
import pytest

from oracle import vit64 as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_00690_amd import vl
    vl.lib()
    return vl


def _oracle_bits(bits_u32: np.ndarray) -> np.ndarray:
    """The oracle's BF16 rounding of the FP32 values with these bit patterns,
    as BF16 bit patterns."""
    r = O.bf16_round(bits_u32.view(np.float32))
    return (r.astype(np.float32).view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def test_bf16_rounding_every_fp32_pattern(V):
    chunk = 1 << 24
    n_chunks = (1 << 32) // chunk
    mism = {0: 0, 1: 0}
    src = torch.empty(chunk, dtype=torch.int32, device="cuda")
    dst = torch.empty(chunk, dtype=torch.int16, device="cuda")
    base = torch.arange(chunk, dtype=torch.int64, device="cuda")

    def check(c, got0, got1):
        bits = (np.arange(chunk, dtype=np.uint64) + np.uint64(c * chunk)).astype(np.uint32)
        want = _oracle_bits(bits)
        nan = ((bits & np.uint32(0x7F800000)) == np.uint32(0x7F800000)) & \
              ((bits & np.uint32(0x007FFFFF)) != 0)
        return (int(np.sum((got0 != want) & ~nan)), int(np.sum((got1 != want) & ~nan)))

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        futs = []

        def drain(limit):
            while len(futs) > limit:            # bounded: at most 16 chunks held
                a, b = futs.pop(0).result()
                mism[0] += a
                mism[1] += b

        for c in range(n_chunks):
            drain(16)
            # bit patterns c * 2^24 .. as int32 (two's complement view of uint32)
            v = base + c * chunk
            src.copy_(torch.where(v >= 2 ** 31, v - 2 ** 32, v).to(torch.int32))
            outs = []
            for method in (0, 1):
                V.vl_bf16_round(src.view(torch.float32), dst, method)
                outs.append(dst.cpu().numpy().view(np.uint16).copy())
            futs.append(ex.submit(check, c, outs[0], outs[1]))
        drain(0)
    _say(f"  bf16 rounding mismatches over 2^32 patterns (NaN excluded): integer {mism[0]}, "
         f"packed instruction {mism[1]}")
    assert mism[0] == 0 and mism[1] == 0


def test_fp8_weight_quantizer_bitexact(V):
    rng = np.random.Generator(np.random.PCG64(78))
    rows, cols = 40, 1000
    w = rng.standard_normal((rows, cols)) * np.exp(rng.uniform(-12, 6, (rows, 1)))
    w[1] = 0.0                                              # all-zero row: scale 1
    # amax 448: scale exactly 1, so these are midpoints of neighbouring e4m3
    # values (ties to even), subnormal-range values and their neighbours
    w[2] = 0.0
    w[2, 0] = 448.0
    ties = [1.0625, -1.1875, 2.125, 2.375, 13 * 2.0 ** -10, -15 * 2.0 ** -10, 120.0, 232.0,
            -296.0, 2.0 ** -10, -(2.0 ** -10), 3 * 2.0 ** -10, 0.0146484375, 416.0, -432.0]
    w[2, 1:1 + len(ties)] = ties
    w[3] = rng.standard_normal(cols) * 1e-38                # FP32 subnormal weights
    w[4, :] = 1.0
    w[4, 7] = -3.0                                          # w / s can exceed 448 by rounding
    w32 = w.astype(np.float32)
    src = torch.from_numpy(w32).cuda()
    codes = torch.empty((rows, cols), dtype=torch.uint8, device="cuda")
    scales = torch.empty(rows, dtype=torch.float32, device="cuda")
    V.vl_fp8_quantize_rows(src, codes, scales)
    torch.cuda.synchronize()
    q, s = O.quantise_fp8_rows(w32)
    want = O.e4m3_code(q)
    got = codes.cpu().numpy()
    zero = (want & 0x7F) == 0
    assert np.array_equal(got[~zero], want[~zero])
    assert np.all((got[zero] & 0x7F) == 0)
    assert np.array_equal(scales.cpu().numpy(), s.astype(np.float32))
