"""The C-ABI library loads and exports every entry point include/spider.h
declares (no GPU needed: nothing here launches device work)."""
import ctypes as ct
import os
import subprocess

import pytest

from paper_2508_12117_amd import spider

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_is_built():
    assert os.path.exists(spider.LIB_PATH), "run __graft_entry__.build() first"


def test_every_declared_function_is_exported():
    names = spider.header_functions()
    assert "spider_grad" in names and "spider_sgld_steps" in names
    lib = ct.CDLL(spider.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding knows every one of them
    assert sorted(spider._SIGS) == names


def test_exports_are_c_symbols():
    out = subprocess.run(["nm", "-D", "--defined-only", spider.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for n in spider.header_functions():
        assert n in exported, n


def test_version_and_null_handling():
    lib = spider.lib()
    assert lib.spider_version() >= 100
    assert lib.spider_last_error(None) == b"null context"
    assert lib.spider_sync(None) == spider.E_INVALID
    lib.spider_destroy(None)
    assert lib.spider_create(None, 0, None) == spider.E_INVALID


def test_create_rejects_a_missing_device():
    h = ct.c_void_p()
    assert spider.lib().spider_create(ct.byref(h), 4096, None) == spider.E_INVALID
    assert not h.value


def test_header_is_plain_c():
    """The header compiles as C99 with no HIP or torch types."""
    src = os.path.join(ROOT, "include", "spider.h")
    text = open(src).read()
    assert "torch" not in text and "hip_runtime" not in text
    res = subprocess.run(["gcc", "-std=c99", "-fsyntax-only", "-x", "c", src],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr


@pytest.mark.parametrize("name,argc", [("spider_grad", 13), ("spider_sgld_steps", 4),
                                       ("spider_moments", 6), ("spider_load_catalog", 3)])
def test_binding_arities(name, argc):
    assert len(spider._SIGS[name][0]) == argc


def test_struct_layouts_match_the_header():
    """The binding's ctypes structures have the header's sizes and offsets."""
    import tempfile
    structs = {"spider_sgld_cfg": spider.SgldCfg, "spider_map_cfg": spider.MapCfg,
               "spider_catalog_desc": spider.CatalogDesc, "spider_net_desc": spider.NetDesc,
               "spider_chainset": spider.ChainSet}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "spider.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe],
                       check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ct.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
