"""The seeded generators: the vector (torch) hash equals the scalar (Python
int) hash bit for bit, and the published splitmix64 finaliser is what both use."""
import torch

import synth


def _splitmix_stream(seed, n):
    """splitmix64 as published: state += golden gamma; output = mix(state)."""
    out, s = [], seed
    for _ in range(n):
        s = (s + 0x9E3779B97F4A7C15) & synth.MASK64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & synth.MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & synth.MASK64
        out.append(z ^ (z >> 31))
    return out


def test_scalar_hash_is_splitmix_stream():
    key = synth.stream_key(7, 3)
    ref = _splitmix_stream(key, 50)
    assert [synth.hash64(7, 3, c) for c in range(50)] == ref
    rng = synth.HostRng(7, 3)
    assert [rng.next64() for _ in range(50)] == ref


def test_vector_hash_matches_scalar():
    ctr = torch.arange(0, 4000, dtype=torch.int64) * 977 + 5
    h = synth.hash64_t(11, 2, ctr)
    for i in range(0, 4000, 37):
        assert int(h[i]) & synth.MASK64 == synth.hash64(11, 2, int(ctr[i]))
    u = synth.uniform_t(h)
    assert u.dtype == torch.float32 and float(u.min()) >= 0 and float(u.max()) < 1
    assert ((u * 2 ** 24) == torch.round(u * 2 ** 24)).all()
    r = synth.randint_t(h, -128, 127)
    assert int(r.min()) >= -128 and int(r.max()) <= 127


def test_beta25_moments():
    lay = synth.brick_layer(3, 0, 256, 64)
    a = lay[..., 3].double()
    # Beta(2,5): mean 2/7, variance 10/392
    assert abs(float(a.mean()) - 2 / 7) < 0.005
    assert abs(float(a.var()) - 10 / 392) < 0.002
    assert (lay[..., :3] <= lay[..., 3:4]).all()


def test_band_equals_full_layer_rows():
    full = synth.brick_layer(3, 5, 40, 30)
    band = synth.brick_layer(3, 5, 40, 30, row0=11, nrows=7)
    assert torch.equal(full[11:18], band)
