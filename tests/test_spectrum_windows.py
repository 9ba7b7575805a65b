"""The shell-spectrum kernel's enumeration, replayed on the host.

The per-plane spectrum kernel gives each wave a window of 64 consecutive
shells and R row groups per window, finds in every row the contiguous kx range
whose shells fall in the window (exact integer bounds), and walks it in chunks
of 64 modes.  This replays that enumeration with the kernel's integer formulas
and checks that every mode of every plane is visited exactly once, by the
window holding its shell, and that the chunks' shells never decrease along the
lanes (what the segmented scan relies on).  The GPU tests compare the kernel's
spectra with the oracle; this pins the index bounds on grids whose shell
counts need one, two and three windows.
"""
import math

import pytest

LANES, WAVES = 64, 16


def shell(k2):
    return (math.isqrt(4 * k2) + 1) // 2


def wav(i, n):
    return i if i < n // 2 else i - n


def visits(nx, ny, nz):
    H = nx // 2 + 1
    nshell = shell((nx // 2) ** 2 + (ny // 2) ** 2 + (nz // 2) ** 2) + 1
    nwin = (nshell + LANES - 1) // LANES
    assert nwin <= WAVES
    R = WAVES // nwin
    seen = {}
    for kz in range(nz):
        izw = wav(kz, nz)
        for wv in range(WAVES):
            win, grp = wv % nwin, wv // nwin
            if grp >= R:
                continue
            s0 = LANES * win
            s1 = min(s0 + LANES - 1, nshell - 1)
            lo2, hi2 = (2 * s0 - 1) ** 2, (2 * s1 + 1) ** 2
            for ky in range(grp, ny, R):
                A = wav(ky, ny) ** 2 + izw * izw
                if 4 * A >= hi2:
                    continue
                kx0 = 0
                if s0 > 0 and lo2 - 4 * A > 0:
                    B = lo2 - 4 * A
                    t = math.isqrt(B)
                    t += t * t < B
                    kx0 = (t + 1) // 2
                kx1 = min(math.isqrt(hi2 - 4 * A - 1) // 2, H - 1)
                for base in range(kx0, kx1 + 1, LANES):
                    shells = [shell(kx * kx + A) for kx in range(base, min(base + LANES, kx1 + 1))]
                    assert shells == sorted(shells)
                    for i, sh in enumerate(shells):
                        assert s0 <= sh <= s1
                        key = (kz, ky, base + i)
                        assert key not in seen
                        seen[key] = sh
    return nshell, nwin, len(seen) == H * ny * nz


@pytest.mark.parametrize("grid", [(16, 16, 16), (12, 24, 16), (128, 128, 4), (256, 16, 4)])
def test_every_mode_once(grid):
    nshell, nwin, complete = visits(*grid)
    assert complete, (grid, nshell, nwin)
