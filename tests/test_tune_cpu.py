"""The tuner's cache file (no GPU needed): entries are written in the form the
library's elbm_tune reads, an existing key is replaced in place of being duplicated,
other lines are kept, and the candidate lists are valid launch configurations."""
import re

import pytest

from paper_1608_06915_amd import tune

# the line form elbm_tune parses: "key": [g, w, x, t, o, p]
C_FORM = re.compile(r'^ *"([^"]{1,255})": \[(-?\d+), (-?\d+), (-?\d+), (-?\d+), (-?\d+), (-?\d+)\]$')


def test_entry_form_matches_the_library_parser():
    line = tune.format_entry("d3s1_10_20", dict(use_graph=10, wg_per_cu=0, xcd_remap=32, threads=256, occupancy=1,
                                                pipeline=0))
    m = C_FORM.match(line)
    assert m and m.group(1) == "d3s1_10_20" and [int(v) for v in m.groups()[1:]] == [10, 0, 32, 256, 1, 0]


def test_write_replaces_the_key_and_keeps_other_lines(tmp_path):
    p = str(tmp_path / "cache.txt")
    with open(p, "w") as fh:
        fh.write('# header\n"d2s1_1_2": [0, 0, 1, 256, 1, 0]\n"d3s1_5_6": [1, 0, 0, 64, 1, 0]\n')
    tune.write_entry(p, "d3s1_5_6", [10, 2, 32, 128, 4, 2], comment="sphere f32")
    tune.write_entry(p, "d3s2_5_6", [10, 0, 1, 128, 1, 0])
    tune.write_entry(p, "d3s1_5_6", [10, 0, 8, 256, 1, 0], comment="sphere f32")
    text = open(p).read().splitlines()
    assert text[0] == "# header"
    assert sum(1 for t in text if t.startswith('"d3s1_5_6"')) == 1
    assert text.count("# sphere f32") == 1
    c = tune.read_cache(p)
    assert c == {"d2s1_1_2": [0, 0, 1, 256, 1, 0], "d3s1_5_6": [10, 0, 8, 256, 1, 0],
                 "d3s2_5_6": [10, 0, 1, 128, 1, 0]}


def test_bad_keys_and_configurations_are_refused(tmp_path):
    with pytest.raises(ValueError):
        tune.write_entry(str(tmp_path / "c.txt"), 'bad"key', [1, 0, 0, 256, 1, 0])
    with pytest.raises(ValueError):
        tune.format_entry("k", [1, 2, 3])


def test_shipped_cache_parses():
    c = tune.read_cache(tune.DEFAULT_CACHE)
    assert len(c) >= 5
    for key, v in c.items():
        assert re.fullmatch(r"d[23]s[0-3](_\d+)+", key)
        assert v[3] in (64, 128, 256) and v[4] in (1, 4) and v[5] in (0, 1, 2) and 0 <= v[0] <= 64


@pytest.mark.parametrize("kind", ["default", "small"])
def test_candidates_are_valid_launches(kind):
    cands = tune.candidates(kind)
    assert len(cands) >= 3
    for c in cands:
        assert set(c) == set(tune.FIELDS)
        assert c["threads"] in (64, 128, 256) and c["occupancy"] in (1, 4) and c["pipeline"] in (0, 1, 2)
        assert 0 <= c["use_graph"] <= 64 and 0 <= c["wg_per_cu"] <= 64 and 0 <= c["xcd_remap"] <= 4096
