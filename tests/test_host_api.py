"""CPU-only checks of the C ABI's host side: exported symbols, launch
geometry, argument validation, tuning defaults, and the serving
scheduler's allocator and admission queue (g++ with sanitizers)."""
import os
import re
import subprocess
import sys

import pytest

import oracle
import paper_2004_13475_amd as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fractal.h")
FAKE0, FAKE1 = 0x10000000, 0x90000000  # never dereferenced: calls fail first


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fractal_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    declared = header_functions()
    assert len(declared) >= 17
    lib = F.load()
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, f"declared in fractal.h but not exported: {missing}"
    assert sorted(F.EXPORTED) == declared


def test_grid_dims_match_lemma2():
    for k in range(0, 21):
        for r in range(0, min(k, 6) + 1):
            assert F.grid_dims(k, r) == oracle.grid_dims(k - r)
    with pytest.raises(F.FractalError) as e:
        F.grid_dims(4, 5)
    assert e.value.code == F.E_INVAL


@pytest.mark.parametrize("args,frag", [
    ((17, 4, 0, 0.2, FAKE0, FAKE1, 1), "level"),
    ((10, 8, 0, 0.2, FAKE0, FAKE1, 1), "tile level"),
    ((16, 0, 0, 0.2, FAKE0, FAKE1, 1), "block level"),
    ((10, 4, 2, 0.2, FAKE0, FAKE1, 1), "rule"),
    ((10, 4, 1, 0.3, FAKE0, FAKE1, 1), "alpha"),
    ((10, 4, 1, float("nan"), FAKE0, FAKE1, 1), "alpha"),
    ((10, 4, 1, 0.0, FAKE0, FAKE1, 1), "alpha"),
    ((10, 4, 0, 0.2, FAKE0, FAKE1, -1), "negative"),
    ((10, 4, 0, 0.2, 0, FAKE1, 1), "null"),
    ((10, 4, 0, 0.2, FAKE0, FAKE0 + 1024, 1), "overlap"),
    ((10, 4, 0, 0.2, FAKE0 + 4, FAKE1, 1), "aligned"),
])
def test_step_validation(args, frag):
    for fn in (F.lambda_step, F.bb_step, F.lambda_step_mfma):
        with pytest.raises(F.FractalError) as e:
            fn(*args, stream=0)
        assert e.value.code == F.E_INVAL
        assert frag in str(e.value)


def test_steps_zero_is_noop_without_device():
    # a valid call with zero steps returns before touching the GPU
    F.lambda_step(10, 4, 0, 0.2, FAKE0, FAKE1, 0, stream=0)
    F.bb_step(10, 4, 1, 0.2, FAKE0, FAKE1, 0, stream=0)


def test_mfma_level_limit():
    with pytest.raises(F.FractalError):
        F.lambda_map_mfma(20, 3, FAKE0, stream=0)
    with pytest.raises(F.FractalError):
        F.lambda_map(40, 3, FAKE0, stream=0)


def test_tuning_defaults_and_validation():
    for k in range(0, 17):
        for rule in (0, 1):
            r, th, order, flags = F.get_tuning(k, rule)
            assert 0 <= r <= min(k, 7) and k - r <= 15
            assert th in (64, 256) and order in (0, 1, 2)
            lds = (0, 1, 2, 3, 9, 11, 17, 19)
            march = tuple(32 | 1 | nt | fuse | st | occ for nt in (0, 2)
                          for fuse in (0, 8, 16, 64, 128) for st in (0, 256, 512, 1024)
                          for occ in (0, 2048))
            block = tuple(4096 | 1 | fuse | nt for nt in (0, 2)
                          for fuse in (0, 8, 16, 64, 128, 8192, 16384, 32768))
            assert flags in lds + march + block, (k, rule, flags)
            if flags & 4096:  # the block engine: 64 x 64 or 128 x 128 tiles
                assert r in (6, 7) and th == 256
            if flags & 32:  # march launches need 16-byte tile rows
                assert (1 << r) * (1 if rule == 0 else 4) >= 16
    # at level 16 (the highest level a tuning covers) both rules default to
    # the block engine on 128 x 128 tiles (two blocks per lane) with 36-step
    # launches; at levels 14 and 15 to 64 x 64 tiles
    for rule in (0, 1):
        r, th, order, flags = F.get_tuning(16, rule)
        assert (r, th) == (7, 256) and flags & 4096 and flags & F.FLAG_FUSE36, rule
    for k in (14, 15):
        for rule in (0, 1):
            assert F.get_tuning(k, rule)[0] == 6 and F.get_tuning(k, rule)[3] & 4096, (k, rule)
    with pytest.raises(F.FractalError):
        F.set_tuning(10, 0, 8, 64, 0)
    with pytest.raises(F.FractalError):
        F.set_tuning(10, 0, 4, 128, 0)
    with pytest.raises(F.FractalError):
        F.step_tuned(0, 10, 0, 0.2, FAKE0, FAKE1, 1, 4, 64, 9, stream=0)
    with pytest.raises(F.FractalError):
        F.step_tuned(0, 10, 0, 0.2, FAKE0, FAKE1, 1, 4, 64, 0, 4, stream=0)
    # march: needs whole segments, 16-byte rows, a lambda or BB map; FUSE8
    # only with march; one fuse flag at a time
    for map_, rule, r, fl in ((0, 0, 4, 32), (0, 0, 3, 33), (2, 0, 4, 33), (0, 0, 4, 1 | 64),
                              (0, 0, 4, 33 | 8 | 64), (0, 0, 4, 33 | 4096), (0, 0, 4, 1 | 2048),
                              (0, 1, 3, 33 | 128),
                              (0, 0, 4, 1 | 128), (0, 0, 4, 1 | 256), (0, 0, 4, 33 | 256 | 512)):
        with pytest.raises(F.FractalError):
            F.step_tuned(map_, 10, rule, 0.2, FAKE0, FAKE1, 1, r, 256, 2, fl, stream=0)
    F.step_tuned(0, 10, 0, 0.2, FAKE0, FAKE1, 0, 4, 256, 2, 33 | 64, stream=0)  # valid, 0 steps
    F.step_tuned(1, 10, 1, 0.2, FAKE0, FAKE1, 0, 2, 256, 0, 33 | 16, stream=0)
    F.step_tuned(0, 10, 0, 0.2, FAKE0, FAKE1, 0, 4, 256, 2, 33 | 64 | 1024, stream=0)
    # stacks: lambda march only in effect; the BB map accepts and ignores them
    F.step_tuned(1, 10, 1, 0.2, FAKE0, FAKE1, 0, 4, 256, 2, 33 | 2 | 64 | 512, stream=0)
    for fl in (1 | 512, 33 | 256 | 1024):  # no march / two stack heights
        with pytest.raises(F.FractalError):
            F.step_tuned(1, 10, 1, 0.2, FAKE0, FAKE1, 1, 4, 256, 2, fl, stream=0)


FAKEW = 0x20000000  # a fake workspace address


def test_tuning_file_round_trip(tmp_path):
    """Tuned launches persist in a text file keyed by device name, level and
    rule: saved, overwritten in the cache, loaded back; lines for other
    devices are skipped; a malformed file is refused and changes nothing."""
    path = tmp_path / "tuning.txt"
    before = {(k, rule): F.get_tuning(k, rule) for k in (12, 13) for rule in (0, 1)}
    tuned = {(12, 0): (5, 256, 2, 32 | 1 | 64 | 2048), (12, 1): (4, 256, 0, 32 | 1 | 64 | 2),
             (13, 0): (6, 256, 2, 32 | 1 | 128 | 256), (13, 1): (3, 64, 1, 1)}
    try:
        for (k, rule), t in tuned.items():
            F.set_tuning(k, rule, *t)
        F.tuning_save(path)
        lines = path.read_text().splitlines()
        assert lines[0].startswith("#")
        for (k, rule) in tuned:
            F.set_tuning(k, rule, *before[(k, rule)])
        F.tuning_load(path)
        for (k, rule), t in tuned.items():
            assert tuple(F.get_tuning(k, rule)) == t
        # another device's entry is skipped; the current device's is taken
        me = next(ln.split("\t")[0] for ln in lines[1:])
        other = tmp_path / "other.txt"
        other.write_text(f"other-device|gfx000\t12\t0\t7\t64\t0\t1\n"
                         f"{me}\t12\t1\t5\t256\t2\t{32 | 1 | 64}\n")
        F.tuning_load(other)
        assert tuple(F.get_tuning(12, 0)) == tuned[(12, 0)]
        assert tuple(F.get_tuning(12, 1)) == (5, 256, 2, 32 | 1 | 64)
        for bad in ("x\t12\t0\t5\n", f"{me}\t12\t0\t9\t256\t2\t1\n",
                    f"{me}\t12\tzero\t5\t256\t2\t1\n", f"{me}\t12\t0\t5\t128\t2\t1\n"):
            p = tmp_path / "bad.txt"
            p.write_text(bad)
            with pytest.raises(F.FractalError) as e:
                F.tuning_load(p)
            assert e.value.code == F.E_INVAL
        assert tuple(F.get_tuning(12, 1)) == (5, 256, 2, 32 | 1 | 64)
        with pytest.raises(F.FractalError) as e:
            F.tuning_load(tmp_path / "missing.txt")
        assert e.value.code == F.E_DEVICE
    finally:
        for (k, rule), t in before.items():
            F.set_tuning(k, rule, *t)


def test_tuning_file_from_environment(tmp_path):
    """FRACTAL_TUNING_FILE is read before a process's first lookup."""
    path = tmp_path / "env_tuning.txt"
    code = ("import sys; sys.path.insert(0, %r); import paper_2004_13475_amd as F; "
            "F.set_tuning(11, 1, 5, 256, 2, 32 | 1 | 64 | 2); F.tuning_save(%r)" % (ROOT, str(path)))
    subprocess.run([sys.executable, "-c", code], check=True)
    code = ("import sys; sys.path.insert(0, %r); import paper_2004_13475_amd as F; "
            "print(tuple(F.get_tuning(11, 1)))" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], check=True, capture_output=True, text=True,
                         env=dict(os.environ, FRACTAL_TUNING_FILE=str(path)))
    assert out.stdout.strip() == str((5, 256, 2, 32 | 1 | 64 | 2))


def test_batch_validation():
    w = dict(work=FAKEW, work_bytes=1 << 20, stream=0)
    with pytest.raises(F.FractalError):
        F.batch_step([(17, 0, 5, 0.2, FAKE0, FAKE1)], **w)
    with pytest.raises(F.FractalError):  # two instances share a buffer
        F.batch_step([(10, 0, 5, 0.2, FAKE0, FAKE1),
                      (10, 0, 5, 0.2, FAKE1, FAKE1 + (1 << 22))], **w)
    with pytest.raises(F.FractalError):  # unknown flag bits are refused
        F.batch_step([(10, 0, 5, 0.2, FAKE0, FAKE1)], tuning=(4, 64, 2, 8), **w)
    with pytest.raises(F.FractalError):  # bad thread count
        F.batch_step([(10, 0, 5, 0.2, FAKE0, FAKE1)], tuning=(4, 128, 2, 0), **w)
    with pytest.raises(F.FractalError) as e:  # short workspace
        F.batch_step([(10, 0, 5, 0.2, FAKE0, FAKE1)], work=FAKEW, work_bytes=16, stream=0)
    assert "workspace" in str(e.value)
    with pytest.raises(F.FractalError):  # null workspace
        F.batch_step([(10, 0, 5, 0.2, FAKE0, FAKE1)], work=0, work_bytes=1 << 20, stream=0)
    with pytest.raises(F.FractalError):  # misaligned workspace
        F.batch_step([(10, 0, 5, 0.2, FAKE0, FAKE1)], work=FAKEW + 8, work_bytes=1 << 20,
                     stream=0)
    with pytest.raises(ValueError):  # a raw workspace address needs its size
        F.batch_step([(10, 0, 5, 0.2, FAKE0, FAKE1)], work=FAKEW, stream=0)
    with pytest.raises(ValueError):  # a raw stream needs an explicit workspace
        F.batch_step([(10, 0, 5, 0.2, FAKE0, FAKE1)], stream=0)
    # stack flags are accepted by batches (and ignored there)
    F.batch_step([(10, 0, 0, 0.2, FAKE0, FAKE1)], tuning=(4, 256, 2, 33 | 64 | 256), **w)
    F.batch_step([], **w)
    F.batch_step([(10, 0, 0, 0.2, FAKE0, FAKE1)], **w)  # no steps: no-op
    # one 48-byte table entry per launch-size list (at most 6) per instance
    assert F.batch_workspace(0) == 0 and F.batch_workspace(1) == 512
    assert F.batch_workspace(65536) == 65536 * 6 * 48
    with pytest.raises(F.FractalError):
        F.batch_workspace(65537)


def _header_prototype(name):
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"\b" + name + r"\s*\(([^)]*)\)", txt)
    assert m, name
    return [a.strip() for a in m.group(1).split(",")]


def test_boundary_signatures():
    """The serving and batch calls take the arguments the boundary names:
    serve_create(arena, bytes, slots, stream, server) with steps per
    iteration a setter of its own, and batch_step with a caller workspace."""
    create = _header_prototype("fractal_serve_create")
    assert [a.split()[-1].lstrip("*") for a in create] == \
        ["d_arena", "arena_bytes", "max_slots", "stream", "server"]
    setter = _header_prototype("fractal_serve_set_steps_per_iter")
    assert [a.split()[-1].lstrip("*") for a in setter] == ["server", "steps_per_iter"]
    batch = _header_prototype("fractal_batch_step")
    assert [a.split()[-1].lstrip("*") for a in batch] == \
        ["inst", "count", "tuning", "d_work", "work_bytes", "stream"]
    assert [a.split()[-1].lstrip("*") for a in _header_prototype("fractal_batch_workspace")] == \
        ["count", "bytes"]


def test_block_engine_validation():
    """The block engine takes 64 x 64 or 128 x 128 tiles (r = 6 or 7) with whole segments and
    256 threads, the lambda or BB map, and no march, stack or occupancy
    flags; 24, 32 and 36 steps per launch only on the block engine; anything
    else is refused before any device work."""
    B = F.FLAG_BLOCK | F.FLAG_SEGMENTS | F.FLAG_FUSE16
    bad = [(0, 0, 12, 5, 256, B),                       # automaton, 32 x 32 tiles
           (0, 1, 12, 5, 256, B),                       # 32 x 32 tiles
           (0, 0, 12, 8, 256, B),                       # 256 x 256 tiles
           (2, 1, 12, 6, 256, B),                       # matrix-core map
           (0, 1, 12, 6, 256, B | F.FLAG_MARCH),
           (0, 1, 12, 6, 256, B | F.FLAG_STACK2),
           (0, 1, 12, 6, 256, B | F.FLAG_OCC_ALT),
           (0, 1, 12, 6, 256, F.FLAG_BLOCK | F.FLAG_FUSE16),  # no whole segments
           (0, 1, 12, 6, 64, B),
           (0, 1, 12, 6, 256, B | F.FLAG_FUSE8),        # two FUSE flags
           (0, 1, 12, 6, 256, B & ~F.FLAG_FUSE16 | F.FLAG_FUSE24 | F.FLAG_FUSE36),
           (0, 1, 12, 4, 256, F.FLAG_MARCH | F.FLAG_SEGMENTS | F.FLAG_FUSE24),  # deep: block only
           (0, 0, 12, 4, 256, F.FLAG_MARCH | F.FLAG_SEGMENTS | F.FLAG_FUSE36),
           (0, 1, 12, 4, 256, F.FLAG_SEGMENTS | F.FLAG_FUSE32)]
    for map_, rule, k, r, th, fl in bad:
        with pytest.raises(F.FractalError) as e:
            F.step_tuned(map_, k, rule, 0.2, FAKE0, FAKE1, 3, r, th, 2, fl, stream=0)
        assert e.value.code == F.E_INVAL, (map_, rule, r, th, fl)
    before, before_ca = F.get_tuning(12, 1), F.get_tuning(12, 0)
    F.set_tuning(12, 1, 6, 256, 2, B)  # accepted as a tuning
    try:
        assert tuple(F.get_tuning(12, 1)) == (6, 256, 2, B)
        F.set_tuning(12, 1, 7, 256, 2, B)  # 128 x 128 tiles, two blocks per lane
        assert tuple(F.get_tuning(12, 1)) == (7, 256, 2, B)
        F.set_tuning(12, 0, 7, 256, 2, B)
        assert tuple(F.get_tuning(12, 0)) == (7, 256, 2, B)
    finally:
        F.set_tuning(12, 1, *before)
        F.set_tuning(12, 0, *before_ca)


def test_reduce_raw_workspace_needs_size():
    with pytest.raises(ValueError):
        F.reduce(0, 10, 4, 0, FAKE0, FAKEW, FAKE1, stream=0)
    with pytest.raises(F.FractalError) as e:  # the library sees the short size
        F.reduce(0, 10, 4, 0, FAKE0, FAKEW, FAKE1, stream=0, work_bytes=8)
    assert "workspace" in str(e.value)
    f = F.nbb_builtin(F.NBB_CARPET)
    with pytest.raises(ValueError):
        F.nbb_reduce(f, 0, 4, 1, FAKE0, FAKEW, FAKE1, stream=0)


def test_serving_scheduler_unit(tmp_path):
    exe = tmp_path / "serve_sched_test"
    src = os.path.join(ROOT, "tests", "serve_sched_test.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-omit-frame-pointer", src, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    assert "serve_sched ok" in out.stdout


@pytest.mark.parametrize("san", [["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                                 ["-fsanitize=thread"]])
def test_serving_core_fake_executor(tmp_path, san):
    """The server's scheduler core against a fake executor and a fake clock:
    budget, FIFO without skip-ahead, slot reuse, iteration sizes, p50/p99
    bookkeeping, failures confined to the requests they touch, and the two
    scheduling threads -- under ASan/UBSan, and under TSan."""
    exe = tmp_path / "serve_core_test"
    src = os.path.join(ROOT, "tests", "serve_core_test.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", *san, "-fno-omit-frame-pointer",
                    "-pthread", "-Wall", "-Wextra", src, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "serve_core ok" in out.stdout
    assert "ThreadSanitizer" not in out.stderr, out.stderr[-4000:]


def test_oracle_and_product_share_nothing():
    """The oracle never imports the GPU package and vice versa."""
    prod = os.path.join(ROOT, "paper_2004_13475_amd")
    for dirpath, _, files in os.walk(prod):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower(), f"{f} mentions the oracle"
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c", ".h")):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2004_13475_amd" not in txt and "csrc" not in txt


def test_compact_sizes_and_validation():
    """Compact storage holds 3^(k-r) tiles of 4^r cells; tile rows must span
    16 bytes, k <= 20, k - r <= 18."""
    for rule, S in ((0, 1), (1, 4)):
        for k in range(0, 21):
            for r in range(0, 8):
                ok = r <= k and k - r <= 18 and (1 << r) * S >= 16
                if ok:
                    assert F.compact_bytes(k, r, rule) == 3 ** (k - r) * 4 ** r * S
                else:
                    with pytest.raises(F.FractalError):
                        F.compact_bytes(k, r, rule)
    with pytest.raises(F.FractalError):
        F.compact_bytes(21, 7, 0)
    # zero steps is a no-op that touches no device memory
    F.compact_step(10, 4, 0, 0.2, FAKE0, FAKE1, 0, 0, stream=0)
    # compact states take the march engine: no 24-, 32- or 36-step launches
    for fl in (F.FLAG_FUSE24, F.FLAG_FUSE32, F.FLAG_FUSE36):
        with pytest.raises(F.FractalError) as e:
            F.compact_step(10, 4, 0, 0.2, FAKE0, FAKE1, 0, fl, stream=0)
        assert e.value.code == F.E_INVAL
