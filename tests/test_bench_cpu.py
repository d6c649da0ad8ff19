"""Host logic of bench.py: the counter summaries under profiles/ are keyed by
a hash of the kernels' code without comments, so a comment edit keeps the
figures valid and any code edit invalidates them (traffic becomes null)."""
import os
import re
import shutil
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture()
def bench_copy(tmp_path, monkeypatch):
    """A copy of the sources and summaries whose hashes are set to match the
    copied code, with bench.py pointed at it."""
    import bench
    csrc = tmp_path / "paper_1204_5072_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("kpz.hip", "kpz_slice.h", "kpz_device.h", "kpz_ring.hip"):
        shutil.copy(os.path.join(ROOT, "paper_1204_5072_amd", "csrc", f), csrc / f)
    shutil.copytree(os.path.join(ROOT, "profiles"), tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    for name, srcs in (("kpz_sweep_L65536_hbm_counters.md", ("kpz.hip", "kpz_slice.h", "kpz_device.h")),
                       ("kpz_ring_L2p30_kernel_trace.md", ("kpz_ring.hip", "kpz_device.h"))):
        p = tmp_path / "profiles" / name
        p.write_text(re.sub(r"code_sha256 = [0-9a-f]{64}",
                            "code_sha256 = " + bench.code_sha256(srcs), p.read_text()))
    return bench, csrc


def test_summaries_carry_a_hash_and_figures():
    text = open(os.path.join(ROOT, "profiles", "kpz_sweep_L65536_hbm_counters.md")).read()
    assert re.search(r"code_sha256 = [0-9a-f]{64}", text)
    for key in ("1024x32", "1024x32,in_place", "1024x32,device_dt"):
        m = re.search(r"traffic_bytes_per_mcs\[%s\] = (\d+)" % re.escape(key), text)
        assert m and int(m.group(1)) > 2 * 2 ** 30   # at least the algorithmic 2 GiB
        m = re.search(r"valu_wave_instr_per_mcs\[%s\] = (\d+)" % re.escape(key), text)
        assert m and int(m.group(1)) > 0


def test_matching_code_gives_the_figures(bench_copy):
    bench, _ = bench_copy
    for block, kw in (((1024, 32), {}), ((1024, 32), {"in_place": True}),
                      ((1024, 32), {"device_dt": True})):
        traffic, valu = bench.sweep_counters(block, **kw)
        assert traffic > 2 * 2 ** 30 and valu > 0
    assert bench.ring_valu_per_mcs() > 0
    assert bench.sweep_counters((1024, 64)) == (None, None)   # not measured


def test_comment_edits_keep_the_figures(bench_copy):
    bench, csrc = bench_copy
    before = bench.sweep_counters((1024, 32))
    p = csrc / "kpz.hip"
    p.write_text("// an added line comment\n/* and a block\n   comment */\n\n" + p.read_text()
                 + "\n// end\n")
    assert bench.sweep_counters((1024, 32)) == before


def test_code_edits_void_the_figures(bench_copy):
    bench, csrc = bench_copy
    p = csrc / "kpz_device.h"
    p.write_text(p.read_text().replace("0x9E3779B9u", "0x9E3779B8u"))
    assert bench.sweep_counters((1024, 32)) == (None, None)
    assert bench.ring_valu_per_mcs() is None
