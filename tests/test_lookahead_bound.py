"""The deep kernels' look-ahead skips a fish's objectives when its move
cannot reach a threshold T: q = fma(dx, dx, RN(dy * dy)) < L(T) must imply
|RN(c - nc)| < T, c and nc being the binary32 objectives before and after the
plain swim (each operation rounded on its own).  Checked here on the CPU in
binary32 numpy arithmetic on adversarial moves: fish at the walls, in the
corners, at the centre, moves at the largest displacement, and thresholds
just above the largest |diff| the moves can make; the limit L is restated
from its derivation (the kernels' comment gives it)."""
import math

import numpy as np

f32 = np.float32


def skip_limit(T: float, H: float, S: float) -> float:
    K = 2.0**-24 * 1.5 * (5.1 * H + S) + 2.0**-60
    root = (T - 2.0**-60) / (1.0 + 2.0**-23) - K
    if not root > 0.0:
        return 0.0
    L = root * root * (1.0 - 2.0**-22)
    Lf = np.float32(L)
    if float(Lf) > L:
        Lf = np.nextafter(Lf, f32(0))
    return float(Lf)


def objective(x, y):
    return np.sqrt(x * x + y * y)  # binary32: each product, the sum and the root rounded


def test_skip_implies_small_change():
    rng = np.random.default_rng(7)
    for H, S in ((100.0, 0.1), (1.0, 0.5), (2.0**40, 3.0), (100.0, 2.0**-20)):
        Hf, Sf = f32(H), f32(S)
        n = 400_000
        # positions: uniform, on the walls, in the corners, near the centre
        x = rng.uniform(-H, H, n).astype(np.float32)
        y = rng.uniform(-H, H, n).astype(np.float32)
        k = n // 8
        x[:k] = Hf * rng.choice([-1, 1], k)
        y[k:2 * k] = Hf * rng.choice([-1, 1], k)
        x[2 * k:3 * k] = Hf * rng.choice([-1, 1], k)
        y[2 * k:3 * k] = Hf * rng.choice([-1, 1], k)
        x[3 * k:4 * k] = rng.uniform(-1e-3, 1e-3, k) * S
        y[3 * k:4 * k] = rng.uniform(-1e-3, 1e-3, k) * S
        # displacements as the kernels form them, many at the extremes
        r = rng.integers(0, 2**24, (2, n), dtype=np.int64)
        r[:, :n // 4] = rng.choice([0, 2**24 - 1], (2, n // 4))
        S23 = f32(Sf * f32(2.0**-23))
        dx = (S23.astype(np.float64) * r[0] - float(Sf)).astype(np.float32)  # exact fma value
        dy = (S23.astype(np.float64) * r[1] - float(Sf)).astype(np.float32)
        nx = np.clip(x + dx, -Hf, Hf)
        ny = np.clip(y + dy, -Hf, Hf)
        diff = np.abs(objective(x, y) - objective(nx, ny)).astype(np.float64)
        q = (dx.astype(np.float64) * dx + (dy * dy).astype(np.float64)).astype(np.float32)
        Ts = [float(np.quantile(diff, p)) for p in (0.5, 0.9, 0.99, 0.999, 0.99999)]
        Ts += [float(diff.max()), S * math.sqrt(2) * 0.99, S * 0.5]
        for T in Ts:
            L = skip_limit(T, H, S)
            skipped = q < f32(L)
            assert skipped.any() or L == 0.0
            assert (diff[skipped] < T).all(), (H, S, T, diff[skipped].max())
