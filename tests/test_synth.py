"""The seeded input generators: shapes and statistics they promise (checked
with the oracle's spectrum, itself pinned by a plain-loop count)."""
import numpy as np

from paper_1003_4322_amd import synth


def test_generator_has_its_target_shell_energies(ref):
    N = 32
    u = synth.random_ns(N, 1, 2.0)
    spec, tot = ref.energy_spectrum(u)
    tgt = synth.target_spectrum(N, 2.0)
    assert np.abs(spec - tgt).max() < 1e-14
    assert abs(tot[0] - 0.5) < 1e-14


def test_mhd_recipe_energies(ref):
    """E_u = E_b = 1/2 for the Elsasser recipe (independent seeds)."""
    z = synth.random_mhd(24, 3, 4, 3.0)
    _, tot = ref.mhd_spectrum(z)
    assert abs(tot[0] - 0.5) < 1e-14 and abs(tot[1] - 0.5) < 1e-14
    assert abs(tot[2]) < 0.2


def test_flat_solenoidal():
    """Solenoidal, zero outside the 2/3 sphere and at k = 0, Hermitian on the
    kx = 0 plane, energy 1/2 per group, and flat: the mean |v|^2 per mode of
    the outermost kept shells is within 10 % of that of the inner ones."""
    N = 24
    v = synth.flat_solenoidal(N, 5, groups=2)
    k = np.where(np.arange(N) < N // 2, np.arange(N), np.arange(N) - N)
    KZ, KY, KX = np.meshgrid(k, k, np.arange(N // 2 + 1), indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    keep = (9 * k2 < N * N) & (k2 > 0)
    for g in range(2):
        u = v[3 * g:3 * g + 3]
        assert np.abs(u[:, ~keep]).max() == 0.0
        assert np.abs(KX * u[0] + KY * u[1] + KZ * u[2]).max() < 1e-15
        p0 = u[:, :, :, 0]
        mirror = p0[:, (-np.arange(N)) % N][:, :, (-np.arange(N)) % N]
        assert np.abs(p0 - np.conj(mirror)).max() < 1e-16
        w = np.where(KX == 0, 1.0, 2.0)
        assert abs(0.5 * np.sum(w * np.sum(np.abs(u) ** 2, axis=0)) - 0.5) < 1e-13
        m2 = np.sum(np.abs(u) ** 2, axis=0)
        s = synth.shell_index(k2)
        inner = m2[keep & (s >= 2) & (s <= 3)].mean()
        outer = m2[keep & (s >= 6)].mean()
        assert abs(outer / inner - 1.0) < 0.1, (inner, outer)
    # groups use different seeds
    assert np.abs(v[:3] - v[3:]).max() > 0.01
