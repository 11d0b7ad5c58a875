"""Host logic of the launch-option table: bucketing, lookup and the
one-variant-per-kernel-family pass."""
from paper_2410_10447_amd import autotune


def _entry(atoms, tpi, rates, variant):
    return {"atoms": atoms, "torsions": 4, "threads_per_ind": tpi, "variant": variant,
            "evals_per_s": rates[f"v{variant}_b{tpi}"], "measured": rates}


def test_bucket_keys_cover_the_size_range():
    keys = set(autotune.all_buckets())
    assert len(keys) == 16
    for n in (1, 12, 32, 33, 64, 65, 100, 128):
        for t in (0, 7, 8, 31, 32):
            assert autotune.bucket(n, t) in keys
    assert autotune.bucket(64, 0) == "a1_t0" and autotune.bucket(65, 0) == "a2_t0"


def test_shipped_table_is_family_consistent():
    t = autotune.load()
    assert set(t["buckets"]) == set(autotune.all_buckets())
    fams = {}
    for e in t["buckets"].values():
        fams.setdefault(autotune.family(e), set()).add(e["variant"])
        assert e["threads_per_ind"] in (64, 128, 256)
    assert all(len(v) == 1 for v in fams.values()), fams


def test_unify_families_within_tolerance():
    table = {"buckets": {
        "a0_t0": _entry(16, 64, {"v0_b64": 100.0, "v1_b64": 99.0}, 0),
        "a0_t1": _entry(16, 64, {"v0_b64": 98.0, "v1_b64": 100.0}, 1),
        "a2_t0": _entry(80, 128, {"v0_b64": 50.0, "v1_b64": 50.0, "v0_b128": 70.0, "v1_b128": 60.0}, 0),
        "a2_t1": _entry(80, 128, {"v0_b64": 50.0, "v1_b64": 50.0, "v0_b128": 60.0, "v1_b128": 70.0}, 1),
    }}
    autotune.unify_families(table, tol=0.03)
    b = table["buckets"]
    # one-slot: variant 1 loses 1 % in a0_t0, variant 0 loses 2 % in a0_t1 -> variant 1
    assert b["a0_t0"]["variant"] == 1 and b["a0_t1"]["variant"] == 1
    assert b["a0_t0"]["evals_per_s"] == 99.0
    # two-wave: either variant loses > 3 % somewhere -> left per bucket
    assert b["a2_t0"]["variant"] == 0 and b["a2_t1"]["variant"] == 1
    assert table["families"]["one-slot"]["unified"] and not table["families"]["two-wave"]["unified"]


def test_candidates_cover_the_tuning_space():
    """Variant x threads per individual (64, 128, 256) x layout for every
    ligand; two individuals per wave only where two fit one wave."""
    small = autotune.candidates(16, 4)
    large = autotune.candidates(48, 4)
    keys_small = {autotune.cand_key(c) for c in small}
    keys_large = {autotune.cand_key(c) for c in large}
    for tpi in (64, 128, 256):
        for v in (0, 1):
            assert f"v{v}_b{tpi}" in keys_large and f"v{v}_b{tpi}_plain" in keys_large
    assert {"v0_b64_x2", "v0_b64_plain_x2"} <= keys_small
    assert not any(k.endswith("_x2") for k in keys_large)
    assert not any(k.endswith("_x2") for k in {autotune.cand_key(c) for c in autotune.candidates(30, 26)})


def test_families_and_choice_of_two_per_wave():
    assert autotune.family({"threads_per_ind": 256, "atoms": 100}) == "four-wave"
    assert autotune.family({"threads_per_ind": 128, "atoms": 40}) == "two-wave"
    assert autotune.family({"threads_per_ind": 64, "atoms": 40, "two_per_wave": True}) == "two-per-wave"
    assert autotune.family({"threads_per_ind": 64, "atoms": 100}) == "two-slot"
    # a bucket that takes two per wave: ligands of the bucket that do not fit
    # (more than 25 torsions) get one wave each
    t = {"buckets": {autotune.bucket(20, 26): {"variant": 0, "threads_per_ind": 64, "plain_maps": False,
                                                 "two_per_wave": True}}}
    path = "/nonexistent/table.json"
    autotune._cache[path] = t
    try:
        assert autotune.choose(20, 24, path)["two_per_wave"]
        assert not autotune.choose(20, 26, path)["two_per_wave"]
    finally:
        autotune._cache.pop(path, None)


def test_shared_launch_variant():
    """The families that can share a launch take one variant on the
    corner-expanded maps when it costs at most 6 % anywhere; with two per
    wave among them, the shuffle (the only reduction two per wave has)."""
    def entry(atoms, tpi, two, rates, variant):
        e = {"atoms": atoms, "torsions": 4, "threads_per_ind": tpi, "variant": variant, "plain_maps": False,
             "measured": rates}
        if two:
            e["two_per_wave"] = True
        e["evals_per_s"] = rates[autotune.cand_key(e)]
        return e
    table = {"buckets": {
        "a0_t0": entry(16, 64, True, {"v0_b64_x2": 100.0, "v0_b64": 60.0, "v1_b64": 61.0}, 0),
        "a1_t0": entry(48, 64, False, {"v0_b64": 97.0, "v1_b64": 100.0}, 1),
        "a2_t0": entry(80, 128, False, {"v0_b128": 99.0, "v1_b128": 100.0, "v0_b64": 80.0}, 1),
    }}
    autotune.unify_shared_launch(table)
    b = table["buckets"]
    assert table["shared_launch"]["unified"] and table["shared_launch"]["variant"] == 0
    assert all(e["variant"] == 0 and not e["plain_maps"] for e in b.values())
    assert b["a1_t0"]["evals_per_s"] == 97.0
    # a loss above the tolerance leaves the buckets alone
    table["buckets"]["a1_t0"] = entry(48, 64, False, {"v0_b64": 90.0, "v1_b64": 100.0}, 1)
    autotune.unify_shared_launch(table)
    assert not table["shared_launch"]["unified"] and table["buckets"]["a1_t0"]["variant"] == 1
