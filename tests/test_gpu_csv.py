"""CSV ingestion on the GPU against the oracle, bit-exact: codes, timestamps,
dictionary byte ranges and counts, on the road-fines fixture, synthetic logs
(ISO ms / ns and integer timestamps), seeded texts with quoted separators,
quotes and newlines (also across 4096-byte tiles), CRLF and blank lines, parse
errors at the same row, capacity, and forced hash collisions."""
import json
import os
import random

import numpy as np
import pytest
import torch

import oracle
from paper_2204_04898_amd import pm4g, synth
from tests.gpu_util import DEV, note

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gpu(text: bytes, *args, **kw):
    t = torch.frombuffer(bytearray(text), dtype=torch.uint8).to(DEV) if text else torch.zeros(0, dtype=torch.uint8,
                                                                                               device=DEV)
    return pm4g.pm4g_ingest_csv(t, *args, **kw)


def _check(text: bytes, cols=(0, 1, 2), sep=b",", has_header=True, ts_iso=False, ts_scale=3):
    g = _gpu(text, *cols, sep=sep, has_header=has_header, ts_iso=ts_iso, ts_scale=ts_scale)
    o = oracle.ingest_csv(text, *cols, sep=sep, has_header=has_header, ts_iso=ts_iso, ts_scale=ts_scale)
    assert (g["n_rows"], g["n_cases"], g["n_acts"]) == (o["n_rows"], o["n_cases"], o["n_acts"])
    assert np.array_equal(g["case_code"].cpu().numpy(), o["case"])
    assert np.array_equal(g["act_code"].cpu().numpy(), o["act"])
    assert np.array_equal(g["ts"].cpu().numpy(), o["ts"])
    for gk, ok in (("case_dict_off", "case_off"), ("case_dict_len", "case_len"), ("act_dict_off", "act_off"),
                   ("act_dict_len", "act_len")):
        assert np.array_equal(g[gk].cpu().numpy(), o[ok]), gk
    return g, o


def test_golden_road_fines():
    gd = json.load(open(os.path.join(GOLDEN, "worked_road_fines.json")))["csv"]
    text = open(os.path.join(GOLDEN, gd["file"]), "rb").read()
    g, _ = _check(text)
    assert g["case_code"].tolist() == gd["case"] and g["act_code"].tolist() == gd["act"]
    assert g["ts"].tolist() == gd["ts"]


@pytest.mark.parametrize("k,scale,unit,iso", [(2, 0.02, "ms", True), (2, 0.02, "ms", False), (3, 0.002, "ns", True)])
def test_synthetic_logs(k, scale, unit, iso):
    log = synth.config_log(k, scale)
    text = synth.log_csv(log, unit, iso)
    note(f"csv: config {k} scale {scale} {unit} iso={iso}: {len(text)} bytes")
    g, o = _check(text, ts_iso=iso, ts_scale=3 if unit == "ms" else 9)
    assert np.array_equal(o["ts"], log.ts)
    # the codes follow first appearance: the first row's case is 0, and so on
    assert g["case_code"][0].item() == 0 and g["act_code"][0].item() == 0


def _field(rng, long_ok):
    alphabet = "ab Z,\"';\t\r\nxé中"
    n = rng.choice([0, 1, 3, 6]) if not (long_ok and rng.random() < 0.05) else rng.randint(3000, 9000)
    return "".join(rng.choice(alphabet) for _ in range(n))


def _quote(v, sep, force):
    if force or any(ch in v for ch in (sep, '"', "\r", "\n")) or v == "":
        return '"' + v.replace('"', '""') + '"'
    return v


def _random_text(seed):
    rng = random.Random(seed)
    sep = rng.choice([",", ";", "\t"])
    ncol = rng.randint(3, 5)
    cols = rng.sample(range(ncol), 3)
    iso = rng.random() < 0.5
    nl = rng.choice(["\n", "\r\n"])
    rows = rng.randint(0, 300)
    pool_c = [_field(rng, False) for _ in range(rng.randint(1, 40))]
    pool_a = [_field(rng, False) for _ in range(rng.randint(1, 10))]
    lines = [sep.join(f"h{i}" for i in range(ncol))] if rng.random() < 0.8 else []
    has_header = bool(lines)
    for _ in range(rows):
        r = [_field(rng, True) for _ in range(ncol)]
        r[cols[0]] = rng.choice(pool_c)
        r[cols[1]] = rng.choice(pool_a)
        if iso:
            r[cols[2]] = (f"{rng.randint(1800, 2200):04d}-{rng.randint(1, 12):02d}-{rng.randint(1, 28):02d}"
                          + rng.choice(["", f"T{rng.randint(0, 23):02d}:{rng.randint(0, 59):02d}:"
                                            f"{rng.randint(0, 59):02d}.{rng.randint(0, 999999):06d}+02:30",
                                        f" {rng.randint(0, 23):02d}:{rng.randint(0, 59):02d}Z"]))
        else:
            r[cols[2]] = str(rng.randint(-(2**63), 2**63 - 1))
        force = rng.random() < 0.3
        lines.append(sep.join(_quote(v, sep, force) for v in r))
        if rng.random() < 0.05:
            lines.append("")
    text = nl.join(lines) + (nl if rng.random() < 0.7 else "")
    return text.encode(), tuple(cols), sep.encode(), has_header, iso


@pytest.mark.parametrize("seed", range(40))
def test_seeded_texts(seed):
    text, cols, sep, has_header, iso = _random_text(seed)
    _check(text, cols=cols, sep=sep, has_header=has_header, ts_iso=iso, ts_scale=6)


@pytest.mark.parametrize("text", [b"", b"case,act,t\n", b"case,act,t", b"\n\n\r\n", b"c,a,t\n1,x,5",
                                  b"c,a,t\r\n1,x,5\r", b"c,a,t\n\n\n1,x,5\n\n"])
def test_edge_texts(text):
    _check(text)


@pytest.mark.parametrize("text,iso,row", [
    (b"c,a,t\n1,x,5\n2,y\n3,z,7\n", False, 1),
    (b"c,a,t\n1,x,2006-02-28\n2,y,2006-02-30\n", True, 1),
    (b"c,a,t\n1,x,2006-01-01 24:00\n", True, 0),
    (b"c,a,t\n1,x,2006-01-01T10:00+01:00x\n", True, 0),
    (b"c,a,t\n1,x,12a\n", False, 0),
    (b"c,a,t\n1,x,9223372036854775808\n", False, 0),
    (b"c,a,t\n1,x,5\n2,\"y,6\n", False, 1),
])
def test_parse_errors(text, iso, row):
    with pytest.raises(oracle.CsvParseError) as e:
        oracle.ingest_csv(text, 0, 1, 2, ts_iso=iso)
    assert e.value.row == row
    with pytest.raises(pm4g.Pm4gError) as g:
        _gpu(text, 0, 1, 2, ts_iso=iso)
    assert g.value.code == pm4g.PM4G_E_PARSE and f"row {row}" in str(g.value)


def test_capacity_and_hash_collisions():
    text = synth.log_csv(synth.config_log(2, 0.002), "ms", True)
    with pytest.raises(pm4g.Pm4gError) as e:
        _gpu(text, 0, 1, 2, ts_iso=True, capacity=100)
    assert e.value.code == pm4g.PM4G_E_CAPACITY
    old = pm4g.load().pm4g_debug_csv_hash_bits(3)     # 8 hash values for thousands of cases
    try:
        _check(text, ts_iso=True)
    finally:
        pm4g.load().pm4g_debug_csv_hash_bits(old)
