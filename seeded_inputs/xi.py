"""Counter-based standard normals for the KL coefficients xi.

Definition (SplitMix64 of Steele, Lea and Flood, 2014, used as a
counter-based generator, followed by the Box-Muller transform):

* ``gamma = 0x9E3779B97F4A7C15``;
  ``mix(z)``: ``z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
  z *= 0x94D049BB133111EB; z ^= z >> 31`` (all mod 2**64).
* The SplitMix64 output number ``i`` for ``seed`` is
  ``mix(seed + (i + 1) * gamma)``.
* Coefficient ``k`` of sample ``s`` on level ``l`` belongs to the normal pair
  ``p = k // 2``; the pair uses the outputs with index
  ``i_w = ((((l << 32) | s) << 8 | p) << 1) | w`` for ``w = 0, 1``.
* ``u1 = ((out_0 >> 11) + 1) * 2**-53`` lies in (0, 1],
  ``u2 = (out_1 >> 11) * 2**-53`` lies in [0, 1).
* ``rad = sqrt(-2 ln u1)``; ``xi[2p] = rad cos(2 pi u2)``,
  ``xi[2p+1] = rad sin(2 pi u2)``.

The GPU library implements the same definition independently; integer parts
agree bit for bit and the transcendental parts to a few ulp.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def xi_index_limits():
    """Largest (level, sample, K) that the index packing supports."""
    return {"level": (1 << 15) - 1, "sample": (1 << 32) - 1, "K": 512}


def _mix(z):
    z = z ^ (z >> np.uint64(30))
    z = z * M1
    z = z ^ (z >> np.uint64(27))
    z = z * M2
    return z ^ (z >> np.uint64(31))


def splitmix64_outputs(seed, idx):
    """SplitMix64 output number ``idx`` (uint64 array) for ``seed``."""
    with np.errstate(over="ignore"):
        s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        return _mix(s + (idx + np.uint64(1)) * GAMMA)


def splitmix64_normals(seed, level, first_sample, n_samples, K):
    """xi[n_samples, K] (float64) for samples first_sample .. first_sample+n-1."""
    lim = xi_index_limits()
    if not (0 <= level <= lim["level"]) or K > lim["K"] or K < 1:
        raise ValueError("level or K outside the generator's index packing")
    if first_sample < 0 or first_sample + n_samples - 1 > lim["sample"]:
        raise ValueError("sample index outside the generator's index packing")
    npair = (K + 1) // 2
    s = np.arange(first_sample, first_sample + n_samples, dtype=np.uint64)[:, None]
    p = np.arange(npair, dtype=np.uint64)[None, :]
    with np.errstate(over="ignore"):
        base = ((((np.uint64(level) << np.uint64(32)) | s) << np.uint64(8)) | p) << np.uint64(1)
        o0 = splitmix64_outputs(seed, base)
        o1 = splitmix64_outputs(seed, base | np.uint64(1))
    u1 = ((o0 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (o1 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    out = np.empty((n_samples, 2 * npair), dtype=np.float64)
    out[:, 0::2] = rad * np.cos(ang)
    out[:, 1::2] = rad * np.sin(ang)
    return np.ascontiguousarray(out[:, :K])
