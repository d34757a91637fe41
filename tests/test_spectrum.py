"""The shell-binned spectrum diagnostic (host-side torch, runs on CPU here):
Parseval's identity and the placement of a single mode."""
import math

import pytest

torch = pytest.importorskip("torch")

from paper_2401_03008_amd.runs import shell_spectrum, spectral_slope  # noqa: E402


def test_single_mode_lands_in_its_shell_and_parseval():
    n = 32
    z, y, x = torch.meshgrid(*(torch.arange(n, dtype=torch.float64) / n,) * 3, indexing="ij")
    f = torch.cos(2 * math.pi * (3 * x + 4 * y))  # |k| = 5
    E = shell_spectrum([f])
    assert int(torch.argmax(E)) + 1 == 5
    # Parseval: sum of the spectrum = mean of f^2 (f has zero mean)
    assert float(E.sum()) == pytest.approx(float((f * f).mean()), rel=1e-12)


def test_slope_of_a_power_law():
    E = [k ** (-5.0 / 3.0) for k in range(1, 40)]
    assert spectral_slope(E, 2, 30) == pytest.approx(-5.0 / 3.0, rel=1e-10)
