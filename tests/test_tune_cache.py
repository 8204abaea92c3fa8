"""The autotuner's JSON cache, through the C ABI with explicit device keys
(no GPU needed): what is stored is what a lookup for the same key returns,
entries merge by key, other keys miss, and a malformed file is an error."""

import json

import pytest


@pytest.fixture(scope="module")
def kb():
    from paper_1902_05320_amd import kbatch
    kbatch.load_library()
    return kbatch


def _tile(kb, **kw):
    t = kb.Tile()
    t.waves_per_simd = kw.get("waves", 2)
    t.steps_per_item = kw.get("steps", 8)
    t.staging = kw.get("staging", kb.STAGING_DIRECT)
    for c, v in kw.get("class_steps", {}).items():
        t.class_steps[c] = v
    for c, v in kw.get("class_threads", {}).items():
        t.class_threads[c] = v
    return t


def test_store_then_lookup_round_trip(kb, tmp_path):
    path = str(tmp_path / "tune.json")
    t = _tile(kb, class_steps={0: 4, 4: 16}, class_threads={7: 32, 4: 1})
    kb.tune_store(path, 1, 1 << 20, t, 1.25, arch="gfx950", rocm="7.2")
    doc = json.load(open(path))
    assert doc["format"] == "kbatch-tune-1"
    keys = sorted(str(e["nb_class"]) for e in doc["entries"])
    assert keys == ["*", "0", "4", "7"]  # launch-wide knobs, then the classes that were set
    assert all(e["batch_class"] == 20 and e["variant"] == "sha3_256" for e in doc["entries"])
    got = kb.tune_lookup(1, 1 << 20, path=path, arch="gfx950", rocm="7.2")
    assert got is not None and got.as_dict() == t.as_dict()
    # the batch class is floor(log2(n)): any n in [2^20, 2^21) hits, others miss
    assert kb.tune_lookup(1, (1 << 21) - 1, path=path, arch="gfx950", rocm="7.2") is not None
    assert kb.tune_lookup(1, 1 << 21, path=path, arch="gfx950", rocm="7.2") is None
    assert kb.tune_lookup(3, 1 << 20, path=path, arch="gfx950", rocm="7.2") is None
    assert kb.tune_lookup(1, 1 << 20, path=path, arch="gfx942", rocm="7.2") is None
    assert kb.tune_lookup(1, 1 << 20, path=path, arch="gfx950", rocm="6.4") is None


def test_entries_merge_by_key(kb, tmp_path):
    path = str(tmp_path / "tune.json")
    kb.tune_store(path, -1, 5000, _tile(kb, waves=1, class_steps={2: 2}), arch="gfx950", rocm="7.2")
    kb.tune_store(path, -1, 5000, _tile(kb, waves=3, class_steps={2: 32}), arch="gfx950", rocm="7.2")
    kb.tune_store(path, 0, 5000, _tile(kb, waves=2), arch="gfx950", rocm="7.2")
    doc = json.load(open(path))
    mixed = [e for e in doc["entries"] if e["variant"] == "mixed"]
    assert len(mixed) == 2  # one launch-wide, one class-2 entry: replaced, not duplicated
    got = kb.tune_lookup(-1, 5000, path=path, arch="gfx950", rocm="7.2")
    assert got.waves_per_simd == 3 and got.class_steps[2] == 32
    assert kb.tune_lookup(0, 5000, path=path, arch="gfx950", rocm="7.2").waves_per_simd == 2


def test_missing_file_is_an_empty_cache(kb, tmp_path):
    assert kb.tune_lookup(1, 100, path=str(tmp_path / "absent.json"), arch="gfx950", rocm="7.2") is None


@pytest.mark.parametrize("text", ["{", "[]", '{"format": "other", "entries": []}',
                                  '{"format": "kbatch-tune-1"}',
                                  '{"format": "kbatch-tune-1", "entries": [{"arch": "gfx950"}]}'])
def test_malformed_file_is_an_error(kb, tmp_path, text):
    path = tmp_path / "bad.json"
    path.write_text(text)
    with pytest.raises(kb.KbError):
        kb.tune_lookup(1, 100, path=str(path), arch="gfx950", rocm="7.2")


def test_key_needs_both_names_or_neither(kb, tmp_path):
    lib = kb.load_library()
    t = _tile(kb)
    rc = lib.keccak_tune_store(str(tmp_path / "t.json").encode(), b"gfx950", None, 1, 10, t, -1.0)
    assert rc == kb.KB_EINVAL
    rc = lib.keccak_tune_store(str(tmp_path / "t.json").encode(), b"gfx950", b"7.2", 9, 10, t, -1.0)
    assert rc == kb.KB_EINVAL  # not a SHA-3 variant or -1
    rc = lib.keccak_tune_store(str(tmp_path / "t.json").encode(), b"gfx950", b"7.2", 1, 0, t, -1.0)
    assert rc == kb.KB_EINVAL  # n == 0


def test_last_tile_starts_as_the_defaults(kb):
    t, cached = kb.last_tile()
    assert not cached and t.waves_per_simd == 0 and list(t.class_threads) == [0] * kb.NB_CLASSES
