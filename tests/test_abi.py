"""The C-ABI library: exported symbols, struct layouts and every host-side
error path (all of them run before any device call, so no GPU is needed)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pms.h")

nat = pytest.importorskip("paper_1403_1313_amd.native",
                          reason="libpms.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pms_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) == 21
    assert sorted(nat.SYMBOLS) == names
    lib = ctypes.CDLL(nat.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header(tmp_path):
    """sizeof/offsetof from the C header compiled by gcc == the ctypes mirrors."""
    prog = tmp_path / "layout.c"
    fields = {
        "pms_instance": ["seqs", "n", "t", "l", "d", "out_motifs", "capacity"],
        "pms_result": ["status", "count", "latency_ms"],
        "pms_config": ["chunk", "wg_waves", "wgs_per_cu", "tail_split", "variant", "filter"],
        "pms_stats": ["kernel_ms", "windows_ms", "seq_visits", "batches", "window_compares",
                      "candidate_slots", "grid", "wg_waves", "chunk", "reruns", "variant",
                      "host_prep_ms", "host_finish_ms", "single_batches", "filtered_batches",
                      "filtered_groups"],
        "pms_dev_instance": ["windows", "out", "out_cap", "n", "nw_stride", "l", "d"],
        "pms_work_item": ["begin", "len", "inst"],
        "pms_dev_state": ["count", "visits", "t_done", "items_left"],
        "pms_dev_counters": ["next_item", "error", "batches", "t_start", "single_batches",
                             "filtered_batches", "filtered_groups"],
        "pms_probe_result": ["lane_ops_per_s", "ms", "sclk_mhz", "lane_ops_per_clk_per_cu",
                             "compute_units"],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pms.h"', "int main(void){"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} size %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st} {f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    prog.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    mirrors = {"pms_instance": nat.Instance, "pms_result": nat.Result, "pms_config": nat.Config,
               "pms_stats": nat.Stats, "pms_dev_instance": nat.DevInstance,
               "pms_work_item": nat.WorkItem, "pms_dev_state": nat.DevState,
               "pms_dev_counters": nat.DevCounters, "pms_probe_result": nat.ProbeResult}
    for line in out.splitlines():
        st, what, val = line.split()
        cls = mirrors[st]
        got = ctypes.sizeof(cls) if what == "size" else getattr(cls, what).offset
        assert got == int(val), (st, what)


def test_decode_status_and_stride():
    assert nat.decode(0, 4) == "AAAA"
    assert nat.decode(0b11100100, 4) == "TGCA"
    assert nat.decode(35797, 8) == "GAGTTCCC"
    for s, txt in [(0, "ok"), (1, "invalid argument"), (2, "output capacity exceeded"),
                   (3, "out of memory"), (4, "device error"), (9, "unknown status")]:
        assert nat.status_string(s) == txt
    P, B = nat.LAYOUT_PLANES, nat.LAYOUT_BITSLICED
    assert nat.window_stride(600, 15, P) == 592
    assert nat.window_stride(600, 11, P) == 592
    assert nat.window_stride(16, 16, P) == 16
    assert nat.window_stride(17, 16, P) == 16
    assert nat.window_stride(32, 16, P) == 32
    assert nat.window_stride(10, 11, P) == 0
    assert nat.window_stride(10, 17, P) == 0
    # bit-sliced: 2l words per group of 32 windows
    assert nat.window_stride(600, 15, B) == 19 * 30
    assert nat.window_stride(600, 11, B) == 19 * 22
    assert nat.window_stride(16, 16, B) == 32
    assert nat.window_stride(47, 16, B) == 32
    assert nat.window_stride(48, 16, B) == 64
    assert nat.window_stride(5, 1, B) == 0
    assert nat.window_stride(5, 2, B) == 4
    assert nat.window_stride(600, 15, 2) == 0


@pytest.mark.parametrize("n,t,l,d", [(0, 10, 4, 1), (65, 10, 4, 1), (3, 10, 0, 0), (3, 10, 17, 1),
                                     (3, 3, 4, 1), (3, 10, 4, -1), (3, 10, 4, 5),
                                     (3, (1 << 17) + 1, 4, 1)])
def test_invalid_shapes(n, t, l, d):
    rows = ["A" * max(min(t, 64), 1)] * max(n, 1)
    arr = (ctypes.c_char_p * len(rows))(*[r.encode() for r in rows])
    out = np.full(8, 0xDEADBEEF, dtype=np.uint32)
    cnt = ctypes.c_uint64(8)
    st = nat.lib().pms_solve(arr, n, t, l, d, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                             ctypes.byref(cnt))
    assert st == nat.PMS_ERR_INVALID and cnt.value == 0
    assert (out == 0xDEADBEEF).all()
    assert nat.last_error()


def test_invalid_pointers_and_bytes():
    lib = nat.lib()
    out = np.full(4, 7, dtype=np.uint32)
    optr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    cnt = ctypes.c_uint64(4)
    assert lib.pms_solve(None, 1, 8, 4, 1, optr, ctypes.byref(cnt)) == nat.PMS_ERR_INVALID
    assert lib.pms_solve(None, 1, 8, 4, 1, optr, None) == nat.PMS_ERR_INVALID
    arr = (ctypes.c_char_p * 2)(b"ACGTACGT", None)
    cnt = ctypes.c_uint64(4)
    assert lib.pms_solve(arr, 2, 8, 4, 1, optr, ctypes.byref(cnt)) == nat.PMS_ERR_INVALID
    assert "NULL" in nat.last_error()
    arr = (ctypes.c_char_p * 1)(b"ACGTACGT")
    cnt = ctypes.c_uint64(4)
    assert lib.pms_solve(arr, 1, 8, 4, 1, None, ctypes.byref(cnt)) == nat.PMS_ERR_INVALID
    for bad in [b"ACGTNCGT", b"ACGT-CGT", b"ACGU ACG", b"ACGT\x00CGT", b"acgtacgx"]:
        arr = (ctypes.c_char_p * 1)(bad)
        cnt = ctypes.c_uint64(4)
        assert lib.pms_solve(arr, 1, 8, 4, 1, optr, ctypes.byref(cnt)) == nat.PMS_ERR_INVALID
        assert cnt.value == 0 and (out == 7).all()
        assert "not A/C/G/T" in nat.last_error()


def test_byte_classification_every_value():
    """Every byte value at an odd position of a 70-byte row: only A/C/G/T in
    either case pass validation, and a rejection names the position."""
    lib = nat.lib()
    out = np.zeros(4, dtype=np.uint32)
    optr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    base = bytearray(b"ACGT" * 17 + b"AC")
    for v in range(256):
        row = bytearray(base)
        row[37] = v
        arr = (ctypes.c_char_p * 1)(bytes(row))
        cnt = ctypes.c_uint64(0)
        st = lib.pms_solve(arr, 1, 70, 4, 1, optr, ctypes.byref(cnt))
        if bytes([v]) in b"ACGTacgt":
            assert st in (nat.PMS_OK, nat.PMS_ERR_DEVICE), v
        else:
            assert st == nat.PMS_ERR_INVALID, v
            assert "byte 37 of sequence 0" in nat.last_error(), v


def test_solve_many_rejects_bad_batches():
    lib = nat.lib()
    res = (nat.Result * 1)()
    assert lib.pms_solve_many(None, 1, res) == nat.PMS_ERR_INVALID
    assert lib.pms_solve_many((nat.Instance * 1)(), -1, res) == nat.PMS_ERR_INVALID
    st, motifs, results = nat.solve_many([(["ACGTNACG"], 4, 1), (["ACGT"], 5, 1)])
    assert st == nat.PMS_ERR_INVALID
    assert [r.status for r in results] == [nat.PMS_ERR_INVALID, nat.PMS_ERR_INVALID]


def test_config_validation():
    before = nat.get_config()
    with pytest.raises(nat.PmsError):
        nat.set_config(chunk=100)
    with pytest.raises(nat.PmsError):
        nat.set_config(chunk=1 << 25)
    with pytest.raises(nat.PmsError):
        nat.set_config(wg_waves=17)
    with pytest.raises(nat.PmsError):
        nat.set_config(tail_split=65)
    assert nat.get_config() == before
    nat.set_config(chunk=4096, wg_waves=2)
    assert nat.get_config()["chunk"] == 4096 and nat.get_config()["wg_waves"] == 2
    nat.set_config(reset=True)
    assert nat.get_config() == {"chunk": 4096, "wg_waves": 4, "wgs_per_cu": 0, "tail_split": 0,
                                "variant": 0, "filter": 0}
    with pytest.raises(nat.PmsError):
        nat.set_config(variant=4)
    with pytest.raises(nat.PmsError):
        nat.set_config(filter=3)


def test_injected_failure_propagates(monkeypatch):
    """PMS_TEST_FAIL_NEXT makes exactly the next valid call fail with that status."""
    monkeypatch.setenv("PMS_TEST_FAIL_NEXT", str(nat.PMS_ERR_NOMEM))
    st, cnt, _ = nat.solve_raw(["ACGTACGT"] * 2, 4, 1)
    assert st == nat.PMS_ERR_NOMEM and cnt == 0
    assert "injected" in nat.last_error()
    st2, _, _ = nat.solve_raw(["ACGTACGT"] * 2, 4, 1)
    assert st2 in (nat.PMS_OK, nat.PMS_ERR_DEVICE)  # the injection was consumed
    monkeypatch.setenv("PMS_TEST_FAIL_NEXT", str(nat.PMS_ERR_DEVICE))
    st, motifs, results = nat.solve_many([(["ACGTACGT"] * 2, 4, 1)])
    assert st == nat.PMS_ERR_DEVICE


def test_no_cpu_fallback_without_gpu():
    """Without a GPU a valid call reports a device error; nothing is computed on the CPU."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, cnt, _ = nat.solve_raw(["ACGTACGT"] * 2, 4, 1)
    assert st == nat.PMS_ERR_DEVICE and cnt == 0


def test_package_import_forms():
    """Both import spellings work in a fresh interpreter."""
    for stmt in ("from paper_1403_1313_amd import native; native.decode(0, 2)",
                 "import paper_1403_1313_amd as p; p.native.decode(0, 2)",
                 "import paper_1403_1313_amd.native as n; n.decode(0, 2)"):
        subprocess.run([__import__("sys").executable, "-c", stmt], cwd=ROOT, check=True)


def test_single_hip_runtime_in_process():
    """Loading the binding before torch still maps exactly one HIP runtime."""
    code = ("import paper_1403_1313_amd.native as n, torch\n"
            "maps = [l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l]\n"
            "print(len(set(maps)))\n")
    out = subprocess.run([__import__("sys").executable, "-c", code], cwd=ROOT, check=True,
                         capture_output=True, text=True).stdout.strip()
    assert out == "1"


def test_solve_ex_rejects_bad_input():
    """pms_solve_ex argument checks run before any device work."""
    st, cnt, _ = nat.solve_ex_raw(["ACGTNACG", "ACGT"], 3, 1)
    assert st == nat.PMS_ERR_INVALID and cnt == 0 and "not A/C/G/T" in nat.last_error()
    st, _, _ = nat.solve_ex_raw(["ACGTXACG", "ACGT"], 3, 1, mask_n=True)
    assert st == nat.PMS_ERR_INVALID and "byte 4 of sequence 0" in nat.last_error()
    st, _, _ = nat.solve_ex_raw(["ACGT", "AC"], 3, 1)
    assert st == nat.PMS_ERR_INVALID and "length of sequence 1" in nat.last_error()
    lib = nat.lib()
    arr = (ctypes.c_char_p * 1)(b"ACGTACGT")
    lens = (ctypes.c_int32 * 1)(8)
    cnt = ctypes.c_uint64(0)
    assert lib.pms_solve_ex(arr, 1, None, 3, 1, 0, None, ctypes.byref(cnt)) == nat.PMS_ERR_INVALID
    assert lib.pms_solve_ex(arr, 1, lens, 3, 1, 4, None, ctypes.byref(cnt)) == nat.PMS_ERR_INVALID
    assert lib.pms_solve_ex(arr, 1, lens, 3, 4, 0, None, ctypes.byref(cnt)) == nat.PMS_ERR_INVALID


def test_solve_ex_sequence_without_windows_is_empty():
    """A sequence with no N-free window: no motifs, status OK, no device work
    (so this holds without a GPU as well)."""
    st, cnt, res = nat.solve_ex_raw(["ACGTACGT", "ACNNGTNA"], 3, 3, mask_n=True, both=True)
    assert st == nat.PMS_OK and cnt == 0 and res.size == 0


def test_solve_intersect_rejects_large_balls():
    """The ball-size limit is checked before any device work."""
    st, cnt, _ = nat.solve_intersect_raw(["ACGT" * 8], 16, 10)
    assert st == nat.PMS_ERR_INVALID and cnt == 0 and "PMS_NBHD_MAX_BALL" in nat.last_error()
    st, _, _ = nat.solve_intersect_raw(["ACGTNACGTACG"], 4, 1)
    assert st == nat.PMS_ERR_INVALID and "not A/C/G/T" in nat.last_error()



def test_probe_rejects_unknown_kinds():
    """pms_valu_probe checks the instruction kind before touching a device:
    every enumerator of pms_probe_op is known to the binding, the values
    around them are refused."""
    text = open(HEADER).read()
    kinds = {name: int(v) for name, v in re.findall(r"\b(PMS_PROBE_[A-Z0-9_]+)\s*=\s*(\d+)", text)}
    assert sorted(kinds.values()) == sorted(nat.PROBE_OPS.values())
    r = nat.ProbeResult()
    for bad in (-1, max(kinds.values()) + 1):
        assert nat._lib.pms_valu_probe(bad, 0, 0, ctypes.byref(r)) == nat.PMS_ERR_INVALID


def test_solve_dev_noalloc_rejects_bad_arguments():
    """pms_solve_dev_noalloc checks pointers and sizes before any device work;
    the scratch limit is published in the header."""
    lib = nat.lib()
    cnt = ctypes.c_uint64(0)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every call below is refused first
    assert lib.pms_solve_dev_noalloc(None, 2, 8, 4, 1, fake, 8, fake, None) == nat.PMS_ERR_INVALID
    assert lib.pms_solve_dev_noalloc(fake, 2, 8, 4, 1, None, 8, fake, None) == nat.PMS_ERR_INVALID
    assert lib.pms_solve_dev_noalloc(fake, 2, 8, 4, 1, fake, 8, None, None) == nat.PMS_ERR_INVALID
    for n, t, l, d in [(0, 8, 4, 1), (65, 8, 4, 1), (2, 3, 4, 1), (2, 8, 17, 1), (2, 8, 4, 5)]:
        assert lib.pms_solve_dev_noalloc(fake, n, t, l, d, fake, 8, fake, None) == nat.PMS_ERR_INVALID
    text = open(HEADER).read()
    assert re.search(r"#define PMS_NOALLOC_SCRATCH_BYTES \(128u << 20\)", text)
    del cnt


def test_shutdown_without_device_work():
    """pms_shutdown before any device work makes no HIP call and succeeds;
    twice in a row as well (the binding also runs it at exit)."""
    code = ("import paper_1403_1313_amd.native as n\n"
            "assert n.shutdown() == 0 and n.shutdown() == 0\n"
            "print('ok')\n")
    out = subprocess.run([__import__("sys").executable, "-c", code], cwd=ROOT, check=True,
                         capture_output=True, text=True).stdout.strip()
    assert out == "ok"


def test_sort_codes():
    """pms_sort_codes (host only): ascending order for both sort paths, and
    its argument checks."""
    rng = np.random.default_rng(5)
    for l, k in [(1, 3), (8, 100), (11, 5000), (16, 20000), (13, 70000)]:
        codes = rng.choice(4 ** l, size=min(k, 4 ** l), replace=False).astype(np.uint32)
        want = np.sort(codes)
        assert np.array_equal(nat.sort_codes(codes, l), want)
    with pytest.raises(nat.PmsError):
        nat.sort_codes(np.array([3, 1 << 10], dtype=np.uint32), 4)
    with pytest.raises(nat.PmsError) as e:
        nat.sort_codes(np.array([5, 5, 1], dtype=np.uint32), 4)
    assert e.value.status == nat.PMS_ERR_DEVICE
    assert nat.lib().pms_sort_codes(None, 0, 4) == nat.PMS_OK
    assert nat.lib().pms_sort_codes(None, 3, 4) == nat.PMS_ERR_INVALID


def test_fill_work_items():
    """pms_fill_work_items (host only): the same records as writing the
    ranges out by hand, the max_items cut, and its argument checks."""
    rec = np.dtype([("begin", "<u8"), ("len", "<u4"), ("inst", "<u4")])
    for begin, count, size, inst, room in [(0, 4 ** 8, 4096, 3, 100), (4096, 1000, 64, 7, 100),
                                           (64, 64 * 37 + 5, 64, 0, 10), (0, 1 << 32, 1 << 31, 1, 9),
                                           (100, 0, 64, 2, 4)]:
        out = np.zeros(room, dtype=rec)
        k = nat.fill_work_items(begin, count, size, inst, out.ctypes.data, room)
        want_begins = np.arange(begin, begin + count, size, dtype=np.uint64)[:room]
        assert k == want_begins.size
        assert np.array_equal(out["begin"][:k], want_begins)
        assert np.array_equal(out["len"][:k],
                              np.minimum(size, begin + count - want_begins).astype(np.uint32))
        assert np.all(out["inst"][:k] == inst) and np.all(out["begin"][k:] == 0)
    assert nat.fill_work_items(0, 10, 0, 0, 0, 0) == -1
    assert nat.fill_work_items(0, 10, 64, 0, 0, 5) == -1
    assert nat.fill_work_items(1, 1 << 32, 64, 0, np.zeros(1, dtype=rec).ctypes.data, 1) == -1


def test_instance_records_both_paths():
    """The batched binding's instance records: the column-wise path for
    (n, t) uint8 arrays gives the same fields and row addresses as writing
    each record in turn (the path for other row types)."""
    rng = np.random.default_rng(9)
    arrays = [rng.integers(65, 70, size=(int(n), int(t)), dtype=np.uint8)
              for n, t in zip(rng.integers(1, 6, 7), rng.integers(5, 40, 7))]
    inst = [(a, 4 + i % 3, i % 2) for i, a in enumerate(arrays)]
    caps = np.array([0, 5, 1, 7, 0, 3, 9], dtype=np.uint64)
    outs = np.arange(7, dtype=np.uint64) * 64 + (1 << 20)
    fast, keep_fast = nat._instance_records(inst, caps, outs)
    slow, keep_slow = nat._instance_records([(list(a), l, d) for a, l, d in inst], caps, outs)
    for name in ("n", "t", "l", "d", "out_motifs", "capacity"):
        assert np.array_equal(fast[name], slow[name]), name
    assert np.all(fast["out_motifs"][caps == 0] == 0)
    for i, a in enumerate(arrays):
        ptrs = np.frombuffer((ctypes.c_uint64 * a.shape[0]).from_address(int(fast["seqs"][i])),
                             dtype=np.uint64)
        assert np.array_equal(ptrs, a.ctypes.data + np.arange(a.shape[0], dtype=np.uint64) * a.shape[1])
        rows = (ctypes.c_char_p * a.shape[0]).from_address(int(slow["seqs"][i]))
        assert list(rows) == [bytes(x) for x in a]
    del keep_fast, keep_slow
