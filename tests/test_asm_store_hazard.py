"""Generated-code check (CPU): no vector-memory store wider than 64 bits has
its data registers rewritten by the very next instruction.

The compiler treats such a rewrite as safe for buffer stores that take a
register offset; on gfx950 it is not: with several blocks per CU the store
wrote the new register contents (the double-precision interleaved tables
of the integral-image writer were not reproducible).  The kernels are
written so that no such pair is emitted; this test compiles every HIP
source to gfx950 assembly and checks the emitted code."""
import concurrent.futures as cf
import os
import re
import shutil
import subprocess

import pytest

from paper_2604_13880_amd import build as B

STORE = re.compile(r"^\s*((?:buffer|global|flat)_store_dwordx[34])\s+(.*)")


def _vgprs(tok: str) -> set:
    m = re.match(r"v\[(\d+):(\d+)\]", tok)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", tok)
    return {int(m.group(1))} if m else set()


def _is_code(line: str) -> bool:
    s = line.strip()
    return bool(s) and not s.startswith((";", ".")) and not s.endswith(":")


def wide_store_rewrites(asm: str):
    """(function, store, next instruction) for every wide store whose data
    registers the next instruction writes."""
    lines = asm.splitlines()
    fn, out = None, []
    for i, line in enumerate(lines):
        if re.match(r"^_Z\S+:", line):
            fn = line.split(":")[0]
        m = STORE.match(line)
        if not m:
            continue
        ops = [o.strip() for o in m.group(2).split(",")]
        data = _vgprs(ops[0] if m.group(1).startswith("buffer") else ops[1])
        k = i + 1
        while k < len(lines) and not _is_code(lines[k]):
            k += 1
        if k >= len(lines):
            continue
        nxt = lines[k].strip().split()
        if len(nxt) < 2 or nxt[0].startswith(("s_", "buffer_store", "global_store", "flat_store", "ds_write")):
            continue
        if _vgprs(nxt[1].rstrip(",")) & data:
            out.append((fn, line.strip(), lines[k].strip()))
    return out


def test_checker_flags_a_rewrite_and_passes_a_gap():
    bad = "_Zk:\n\tbuffer_store_dwordx4 v[22:25], v71, s[12:15], s40 offen\n\tv_add_f64 v[22:23], v[8:9], v[12:13]\n"
    ok = "_Zk:\n\tbuffer_store_dwordx4 v[22:25], v71, s[12:15], s40 offen\n\ts_nop 0\n\tv_add_f64 v[22:23], v[8:9], v[12:13]\n"
    narrow = "_Zk:\n\tbuffer_store_dwordx2 v[22:23], v71, s[12:15], s40 offen\n\tv_add_f64 v[22:23], v[8:9], v[12:13]\n"
    other = "_Zk:\n\tglobal_store_dwordx4 v[4:5], v[0:3], off\n\tv_add_u32_e32 v6, 1, v7\n"
    assert len(wide_store_rewrites(bad)) == 1
    assert wide_store_rewrites(ok) == []
    assert wide_store_rewrites(narrow) == []
    assert wide_store_rewrites(other) == []


@pytest.mark.skipif(not shutil.which(B.HIPCC) and not os.path.exists(B.HIPCC), reason="hipcc not available")
def test_no_wide_store_data_rewritten_by_the_next_instruction(tmp_path):
    srcs = [s for s in B.SOURCES if s.endswith(".hip")]

    def asm(src):
        out = tmp_path / (src + ".s")
        r = subprocess.run([B.HIPCC, *B.FLAGS, "--cuda-device-only", "-S", os.path.join(B.CSRC, src), "-o", str(out)],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return src, out.read_text()

    with cf.ThreadPoolExecutor(4) as ex:
        texts = list(ex.map(asm, srcs))
    bad = [(src, *hit) for src, text in texts for hit in wide_store_rewrites(text)]
    assert not bad, bad[:5]
