"""The binding's ctypes structs and record dtypes match the C header's layout:
a small C program built with gcc against the header prints every field's
offset and every struct's size, which must equal what ctypes computes."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2204_04898_amd import pm4g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "pm4g_log": pm4g._Log,
    "pm4g_prepared": pm4g._Prepared,
    "pm4g_dfg_out": pm4g._DfgOut,
    "pm4g_variants_out": pm4g._VarOut,
    "pm4g_batched_out": pm4g._BatchedOut,
    "pm4g_batched_tuning": pm4g.BatchedTuning,
    "pm4g_case_filter": pm4g.CaseFilter,
    "pm4g_efg_out": pm4g._EfgOut,
    "pm4g_csv_schema": pm4g.CsvSchema,
    "pm4g_csv_out": pm4g._CsvOut,
    "pm4g_parquet_schema": pm4g.ParquetSchema,
}
VIEW_FIELDS = ("case_lo", "case_hi", "t_lo", "t_hi")


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pm4g.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append(f'printf("{name} . %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines.append('printf("pm4g_view . %zu\\n", sizeof(pm4g_view));')
    for f in VIEW_FIELDS:
        lines.append(f'printf("pm4g_view {f} %zu\\n", offsetof(pm4g_view, {f}));')
    lines += ["return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    lay = {}
    for ln in out.splitlines():
        s, f, v = ln.split()
        lay[(s, f)] = int(v)
    return lay


@pytest.mark.parametrize("name", sorted(STRUCTS))
def test_ctypes_struct_matches_header(c_layout, name):
    cls = STRUCTS[name]
    assert ctypes.sizeof(cls) == c_layout[(name, ".")], name
    for f, _ in cls._fields_:
        assert getattr(cls, f).offset == c_layout[(name, f)], (name, f)


def test_view_record_matches_header(c_layout):
    dt = np.dtype([("lo", "<i4"), ("hi", "<i4"), ("t_lo", "<i8"), ("t_hi", "<i8")])
    assert dt.itemsize == c_layout[("pm4g_view", ".")]
    for (npf, _), cf in zip(dt.descr, VIEW_FIELDS):
        assert dt.fields[npf][1] == c_layout[("pm4g_view", cf)], cf
