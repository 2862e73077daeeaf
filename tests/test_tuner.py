"""The autotuner's cache on the CPU (no device needed): key format and token buckets,
entries, the nearest-bucket lookup a product call uses, the JSON file (round trip,
entries of another device skipped, malformed files refused with the tuner unchanged)."""

import json

import pytest

from paper_2505_07329_amd import rlwe as r


def sched(method=1, tt=3, order=0, launch=0, ms=1.0):
    return dict(method=method, tt_log2=tt, order=order, launch=launch, ms=ms)


def test_keys_and_buckets():
    assert r.rlwe_tune_key(4096, 2, 2048, 2048, 1, False, 128) == "N4096.P2.K2048.M2048.n1.r0.T128"
    assert r.rlwe_tune_key(4096, 2, 512, 2048, 8, True, 100).endswith(".n8.r1.T128")
    for T, b in ((1, 1), (2, 2), (3, 4), (16, 16), (17, 32), (512, 512), (513, 1024)):
        assert r.rlwe_tune_key(4096, 2, 1, 1, 1, False, T).endswith(f".T{b}")


def test_put_get_and_errors():
    t = r.rlwe_tuner_create("dev")
    k = r.rlwe_tune_key(4096, 2, 2048, 512, 1, False, 16)
    r.rlwe_tuner_put(t, k, sched(ms=2.5))
    got = r.rlwe_tuner_get(t, k)
    assert got["tt_log2"] == 3 and abs(got["ms"] - 2.5) < 1e-6
    with pytest.raises(r.RlweError):
        r.rlwe_tuner_get(t, r.rlwe_tune_key(4096, 2, 2048, 512, 1, False, 32))
    with pytest.raises(r.RlweError):
        r.rlwe_tuner_put(t, "not a key", sched())
    with pytest.raises(r.RlweError):
        r.rlwe_tuner_put(t, k, sched(tt=6))  # at most 32 tokens per workgroup
    with pytest.raises(r.RlweError):
        r.rlwe_tuner_put(t, k, sched(launch=2))
    assert r.rlwe_tuner_size(t) == 1
    r.rlwe_tuner_destroy(t)


def test_lookup_takes_the_nearest_bucket_of_the_same_shape():
    t = r.rlwe_tuner_create("dev")
    shape = (4096, 2, 2048, 2048, 1, False)
    r.rlwe_tuner_put(t, r.rlwe_tune_key(*shape, 16), sched(tt=1, ms=1))
    r.rlwe_tuner_put(t, r.rlwe_tune_key(*shape, 256), sched(tt=4, ms=2))
    assert r.rlwe_tuner_lookup(t, *shape, 16)["tt_log2"] == 1     # exact
    assert r.rlwe_tuner_lookup(t, *shape, 20)["tt_log2"] == 1     # bucket 32: 16 is nearer
    assert r.rlwe_tuner_lookup(t, *shape, 64)["tt_log2"] == 4     # bucket 64: tie, the larger
    assert r.rlwe_tuner_lookup(t, *shape, 4000)["tt_log2"] == 4
    assert r.rlwe_tuner_lookup(t, 4096, 2, 2048, 512, 1, False, 16) is None  # other M
    assert r.rlwe_tuner_lookup(t, 4096, 2, 2048, 2048, 1, True, 16) is None  # raw output
    assert r.rlwe_tuner_lookup(t, 4096, 2, 2048, 2048, 2, False, 16) is None  # packed rows
    r.rlwe_tuner_destroy(t)


def test_json_round_trip_and_device(tmp_path):
    t = r.rlwe_tuner_create("gfx950|MI355X|256")
    keys = [r.rlwe_tune_key(4096, 2, K, M, 1, False, T) for K, M, T in
            ((2048, 2048, 128), (512, 2048, 8), (8192, 2048, 256))]
    for i, k in enumerate(keys):
        r.rlwe_tuner_put(t, k, sched(method=i % 2, tt=i, order=i % 2, launch=1 - i % 2, ms=0.5 + i))
    path = str(tmp_path / "tune.json")
    r.rlwe_tuner_save(t, path)
    doc = json.load(open(path))
    assert doc["device"] == "gfx950|MI355X|256" and len(doc["entries"]) == 3
    t2 = r.rlwe_tuner_create("gfx950|MI355X|256")
    assert r.rlwe_tuner_load(t2, path) == 3
    for k in keys:
        assert r.rlwe_tuner_get(t2, k) == r.rlwe_tuner_get(t, k)
    other = r.rlwe_tuner_create("gfx942|MI300X|304")
    assert r.rlwe_tuner_load(other, path) == 0 and r.rlwe_tuner_size(other) == 0
    for x in (t, t2, other):
        r.rlwe_tuner_destroy(x)


@pytest.mark.parametrize("text", [
    "", "{", '{"device": "d"}', '{"device": "d", "entries": [{"key": "x"}]}',
    '{"device": "d", "entries": [{"key": "N4096.P2.K1.M1.n1.r0.T1", "method": 1, "tt_log2": 9, '
    '"order": 0, "launch": 0, "ms": 1}]}',
    '{"device": "d", "entries": [] ', '["d"]',
])
def test_malformed_files_are_refused(tmp_path, text):
    path = tmp_path / "bad.json"
    path.write_text(text)
    t = r.rlwe_tuner_create("d")
    k = r.rlwe_tune_key(4096, 2, 2048, 2048, 1, False, 1)
    r.rlwe_tuner_put(t, k, sched())
    with pytest.raises(r.RlweError) as ei:
        r.rlwe_tuner_load(t, str(path))
    assert ei.value.code == r.RLWE_EINVAL
    assert r.rlwe_tuner_size(t) == 1 and r.rlwe_tuner_get(t, k)["tt_log2"] == 3
    with pytest.raises(r.RlweError):
        r.rlwe_tuner_load(t, str(tmp_path / "missing.json"))
    r.rlwe_tuner_destroy(t)


def test_mutated_files_load_whole_or_are_refused(tmp_path):
    """Seeded byte mutations of a valid cache file (flipped and inserted bytes, cut
    ranges, truncation): each load either succeeds or raises RLWE_EINVAL with the tuner
    unchanged; none crashes the process."""
    import random
    t = r.rlwe_tuner_create("d")
    for i, (K, M, T) in enumerate(((2048, 2048, 128), (512, 2048, 8), (8192, 2048, 256))):
        r.rlwe_tuner_put(t, r.rlwe_tune_key(4096, 2, K, M, 1, False, T), sched(tt=i, ms=1.0 + i))
    good = str(tmp_path / "good.json")
    r.rlwe_tuner_save(t, good)
    r.rlwe_tuner_destroy(t)
    src = open(good, "rb").read()
    rng = random.Random(7)
    path = tmp_path / "m.json"
    refused = 0
    for _ in range(400):
        b = bytearray(src)
        for _ in range(rng.randint(1, 6)):
            if not b:
                break
            pos, op = rng.randrange(len(b)), rng.random()
            if op < 0.4:
                b[pos] = rng.randrange(256)
            elif op < 0.6:
                del b[pos:pos + rng.randint(1, 30)]
            elif op < 0.85:
                b[pos:pos] = bytes(rng.choice(b'{}[]":,0123456789-eE.') for _ in range(rng.randint(1, 8)))
            else:
                del b[pos:]
        path.write_bytes(bytes(b))
        u = r.rlwe_tuner_create("d")
        k = r.rlwe_tune_key(4096, 2, 1, 1, 1, False, 1)
        r.rlwe_tuner_put(u, k, sched(tt=5))
        try:
            n = r.rlwe_tuner_load(u, str(path))
            assert 0 <= n <= 3 and r.rlwe_tuner_size(u) == 1 + n
        except r.RlweError as e:
            refused += 1
            assert e.code == r.RLWE_EINVAL and r.rlwe_tuner_size(u) == 1
        r.rlwe_tuner_destroy(u)
    assert refused > 300
