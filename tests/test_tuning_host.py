"""Host side of the tile autotuner: the tile classes and the JSON table reader (no GPU)."""
import json
import os

import pytest


@pytest.fixture(scope="module")
def ih():
    from paper_1912_03278_amd import ihmc
    if not os.path.exists(ihmc.LIB_PATH):
        from paper_1912_03278_amd import build
        build.build()
    return ihmc


def test_tile_shapes(ih):
    assert ih.tile_class_count(2) == 3 and ih.tile_class_count(3) == 4
    assert [ih.tile_shape(2, c) for c in range(3)] == [(64, 16, 1), (16, 16, 1), (32, 32, 1)]
    assert [ih.tile_shape(3, c) for c in range(4)] == [(32, 8, 4), (16, 16, 4), (32, 8, 8), (16, 16, 8)]
    for nd, c in ((2, 3), (3, 4), (2, -1)):
        with pytest.raises(ih.IhmcError):
            ih.tile_shape(nd, c)
    with pytest.raises(ih.IhmcError):
        ih.tile_class_count(1)


def entry(**kw):
    e = {"precision": 4, "ndim": 2, "L": [64, 64, 1], "site_field": 0, "class": 1, "source": 1,
         "ns_per_site": [0.01, 0.02, None]}
    e.update(kw)
    return e


def write(tmp_path, doc, name="t.json"):
    p = tmp_path / name
    p.write_text(doc if isinstance(doc, str) else json.dumps(doc))
    return str(p)


def table(*entries):
    return {"format": "ihmc-tile-classes", "version": 1, "entries": list(entries)}


def test_valid_tables(ih, tmp_path):
    assert ih.check_tuning(write(tmp_path, table())) == 0
    doc = table(entry(), entry(ndim=3, L=[17, 17, 17], **{"class": 1}), entry(precision=8, site_field=1, source=2))
    assert ih.check_tuning(write(tmp_path, doc)) == 3
    # an equal key given twice counts once (the later entry wins)
    assert ih.check_tuning(write(tmp_path, table(entry(), entry(**{"class": 2})))) == 1
    # unknown fields are ignored; ns_per_site may be absent
    e = entry(extra="x")
    del e["ns_per_site"]
    assert ih.check_tuning(write(tmp_path, table(e))) == 1


@pytest.mark.parametrize("bad", [
    "not json",
    '{"format": "ihmc-tile-classes", "entries": []} trailing',
    json.dumps({"format": "other", "entries": []}),
    json.dumps({"format": "ihmc-tile-classes"}),
    json.dumps(table(entry(**{"class": 3}))),                    # 2D has classes 0..2
    json.dumps(table(entry(ndim=3, L=[16, 16, 16], **{"class": 4}))),  # 3D has 0..3
    json.dumps(table(entry(L=[2, 64, 1]))),                      # L >= 3
    json.dumps(table(entry(L=[64, 64, 4]))),                     # 2D has L2 = 1
    json.dumps(table(entry(L=[64, 64]))),
    json.dumps(table(entry(precision=2))),
    json.dumps(table(entry(source=0))),                          # rule entries are not stored
    json.dumps(table(entry(site_field=2))),
    json.dumps(table(entry(**{"class": 1.5}))),
    "[" * 40 + "]" * 40,
])
def test_malformed_tables_are_rejected(ih, tmp_path, bad):
    with pytest.raises(ih.IhmcError) as e:
        ih.check_tuning(write(tmp_path, bad))
    assert e.value.code == -1


def test_missing_file(ih, tmp_path):
    with pytest.raises(ih.IhmcError):
        ih.check_tuning(str(tmp_path / "absent.json"))
