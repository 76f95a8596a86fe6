"""Host checks of the error bounds the matrix-core distance pass relies on.

The pass forms x.y from bfloat16 operands: BF16 takes hi.hi' with hi = RNE_bf16(x); BF16x3 takes
hi.hi' + hi.lo' + lo.hi' with lo = RNE_bf16(x - hi).  Its per-row bound charges these forms
kUbf1 (resp. kUbf3) times sum_k |x_k||y_k|.  Here the split is emulated bit for bit on the host
(round-to-nearest-even of the float32 pattern), the products are summed exactly enough in float64,
and the constants compiled into the kernel source are checked to cover adversarial rows: every
element placed where the neglected terms are largest, all signs aligned."""
import os
import re

import numpy as np

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_1710_03013_amd", "csrc", "k_mfma.hip")


def _const(name):
    m = re.search(rf"constexpr float {name} = ([0-9.eE+-]+)f;", open(SRC).read())
    assert m, name
    return float(m.group(1))


def bf16_rne(x):
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def split(x):
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_rne(x)
    lo = bf16_rne((x - hi).astype(np.float32))     # x - hi is exact in float32
    return hi.astype(np.float64), lo.astype(np.float64)


def _errors(x, y):
    x = np.asarray(x, dtype=np.float32)
    y = np.asarray(y, dtype=np.float32)
    hx, lx = split(x)
    hy, ly = split(y)
    exact = np.dot(x.astype(np.float64), y.astype(np.float64))
    scale = np.dot(np.abs(x.astype(np.float64)), np.abs(y.astype(np.float64)))
    e1 = abs(np.dot(hx, hy) - exact) / scale
    e3 = abs(np.dot(hx, hy) + np.dot(hx, ly) + np.dot(lx, hy) - exact) / scale
    return e1, e3


def _adversarial(rng, n):
    """Elements x = 2^e (1 + t): t just under half a bfloat16 ulp (x still rounds down to 2^e), with
    the remainder lo as large as a bfloat16 below 2^-8 and the last remainder r just under half an
    ulp of lo: lo.lo', hi.r' and r.hi' all near their maxima and of one sign."""
    t = np.float64(2.0 ** -8 - 2.0 ** -17 - 2.0 ** -23)
    e = rng.integers(-6, 7, size=n)
    return (2.0 ** e * (1.0 + t)).astype(np.float32)


def test_split_bf16_bounds_cover_adversarial_rows():
    kub1, kub3 = _const("kUbf1"), _const("kUbf3")
    u = 2.0 ** -8
    # the constants are the derived bounds u(2 + u) and 3 u^2 (1 + 2^-7), rounded up
    assert kub1 >= u * (2 + u) and kub1 < u * (2 + u) * (1 + 1e-6)
    assert kub3 >= 3 * u * u * (1 + 2.0 ** -7) and kub3 < 3 * u * u * (1 + 2.0 ** -7) * (1 + 1e-4)
    rng = np.random.default_rng(0)
    worst1 = worst3 = 0.0
    for _ in range(50):
        for d in (16, 64, 128):
            x, y = _adversarial(rng, d), _adversarial(rng, d)
            e1, e3 = _errors(x, y)
            worst1, worst3 = max(worst1, e1), max(worst3, e3)
    # the adversarial rows come close to the true supremum of the split (about 2 u^2) ...
    assert worst3 > 0.95 * 2.0 ** -15
    # ... and the charged constants cover them
    assert worst3 <= kub3 and worst1 <= kub1


def test_split_bf16_bounds_on_random_and_midpoint_rows():
    kub1, kub3 = _const("kUbf1"), _const("kUbf3")
    rng = np.random.default_rng(1)
    for trial in range(300):
        d = int(rng.choice([16, 32, 64, 128]))
        if trial % 3 == 0:      # values on bfloat16 rounding midpoints, mixed signs
            m = 1.0 + (rng.integers(0, 128, size=d) + 0.5) / 128.0
            x = (m * 2.0 ** rng.integers(-4, 5, size=d) * rng.choice([-1, 1], size=d)).astype(np.float32)
            y = (m[::-1] * 2.0 ** rng.integers(-4, 5, size=d)).astype(np.float32)
        else:
            x = rng.normal(scale=10.0, size=d).astype(np.float32)
            y = rng.normal(scale=10.0, size=d).astype(np.float32)
        e1, e3 = _errors(x, y)
        assert e1 <= kub1 and e3 <= kub3


def test_bf16_rne_emulation_matches_torch():
    """The host emulation rounds like torch's float32 -> bfloat16 conversion (round to nearest even)."""
    torch = __import__("pytest").importorskip("torch")
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(scale=100.0, size=4000),
                        (1.0 + (np.arange(256) + 0.5) / 128.0)]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(bf16_rne(x), want)
