"""C-ABI checks that need no GPU: symbols, supported sizes, the host-side
schedule compiler (checked against the oracle's schedule) and validation."""

import os
import re

import pytest

from oracle import mpr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spr.h")


def _lib():
    from paper_2409_07413_amd import binding
    return binding, binding.load()


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(spr_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    binding, lib = _lib()
    names = header_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(binding.EXPORTS)


def test_supported_sizes():
    _, lib = _lib()
    for n in (8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024):
        assert lib.spr_supported_size(n) == 1
    for n in (0, 7, 10, 20, 100, 1000, 1536, 2048, -8):
        assert lib.spr_supported_size(n) == 0


PLAIN = dict(alg=1, G=10, j=16, j_er=4, j_end=0, beta=0.9, chi=0.5, sigma=2.0, sigma_end=1.0,
             tau=0.1, tau_end=0.1)


def test_plain_schedule_matches_oracle_schedule():
    binding, _ = _lib()
    ops = binding.sched_plain(**PLAIN).ops()
    exp = []
    for g in range(1, 11):
        jg, jer, sg, tg = mpr.schedule_at(g, 10, 16, 4, 0, 2.0, 1.0, 0.1, 0.1)
        if jg:
            exp.append((binding.OP_HIO, jg))
        if jer:
            exp.append((binding.OP_ER, jer))
        exp.append((binding.OP_SHRINKWRAP, sg, tg))
    exp.append((binding.OP_GET_ERROR,))
    got = []
    for o in ops:
        if o.kind in (binding.OP_HIO, binding.OP_ER):
            got.append((o.kind, o.count))
            assert o.chi == 0.5
        elif o.kind == binding.OP_SHRINKWRAP:
            got.append((o.kind, o.sigma, o.tau))
        else:
            got.append((o.kind,))
    assert got == exp


MPR = dict(alg=2, G=20, R=3, j=16, j_er=4, j_end=0, j_eval=40, t_min=4, t_max=64, gen_first=1,
           gen_count=0, init_error=1, beta=0.9, chi=0.5, sigma=2.0, sigma_end=0.5, tau=0.1,
           tau_end=0.1 * 2 / 3, c_p=0.6, c_w=0.4)


def test_mpr_schedule_structure_and_iteration_count():
    binding, _ = _lib()
    ops = binding.sched_mpr(**MPR).ops()
    assert ops[0].kind == binding.OP_GET_ERROR and ops[0].scope == binding.SCOPE_PARENTS
    gens = [o for o in ops if o.kind == binding.OP_CROSSOVER]
    assert [o.gen for o in gens] == list(range(1, 21))
    # per generation: R (j + j_ER) + j_eval = 100 iterations on every member
    per_gen = {}
    g = 0
    for o in ops:
        if o.kind == binding.OP_CROSSOVER:
            g = o.gen
        if o.kind in (binding.OP_ER, binding.OP_RAAR):
            per_gen[g] = per_gen.get(g, 0) + o.count
            assert o.scope == binding.SCOPE_ALL
    assert all(v == 100 for v in per_gen.values()) and len(per_gen) == 20
    # order inside a generation follows Alg. mpr / Alg. improve
    seq = []
    for o in ops[1:]:
        if o.kind == binding.OP_CROSSOVER and o.gen == 2:
            break
        seq.append(o.kind)
    K = binding
    assert seq == [K.OP_CROSSOVER, K.OP_STATS, K.OP_RAAR, K.OP_ER, K.OP_SHRINKWRAP, K.OP_RAAR, K.OP_ER,
                   K.OP_SUPPORT_AREA, K.OP_RAAR, K.OP_ER, K.OP_SUPPORT_AREA, K.OP_ER, K.OP_GET_ERROR,
                   K.OP_SHRINKWRAP, K.OP_SELECT]
    areas = [o.which for o in ops if o.kind == binding.OP_SUPPORT_AREA][:2]
    assert areas == [binding.AREA_BEST, binding.AREA_EVAL]
    # linear schedules agree with the oracle at every generation
    g = 0
    for o in ops:
        if o.kind == binding.OP_CROSSOVER:
            g = o.gen
            jg, jer, sg, tg = mpr.schedule_at(g, 20, 16, 4, 0, 2.0, 0.5, 0.1, 0.1 * 2 / 3)
        if o.kind == binding.OP_RAAR:
            assert o.count == jg and abs(o.beta - 0.9) < 1e-15
        if o.kind == binding.OP_SHRINKWRAP:
            assert o.sigma == sg and o.tau == tg
    stats = [o for o in ops if o.kind == binding.OP_STATS]
    assert all(o.gens == 20 for o in stats)


def test_mpr_schedule_resume_window():
    binding, _ = _lib()
    ops = binding.sched_mpr(**dict(MPR, gen_first=7, gen_count=3, init_error=0)).ops()
    assert [o.gen for o in ops if o.kind == binding.OP_CROSSOVER] == [7, 8, 9]
    assert ops[0].kind == binding.OP_CROSSOVER


@pytest.mark.parametrize("bad", [dict(G=0), dict(R=1), dict(alg=3), dict(j=-1)])
def test_mpr_schedule_validation(bad):
    binding, _ = _lib()
    with pytest.raises(binding.SprError) as e:
        binding.sched_mpr(**dict(MPR, **bad))
    assert e.value.code == -1


def test_op_validation():
    binding, _ = _lib()
    for o in (binding.op(binding.OP_HIO, count=3, beta=1.5),
              binding.op(binding.OP_SHRINKWRAP, sigma=9.0, tau=0.1),
              binding.op(binding.OP_SHRINKWRAP, sigma=1.0, tau=2.0),
              binding.op(binding.OP_STATS, gen=0, gens=10),
              binding.op(99),
              binding.op(binding.OP_ER, count=1, scope=5)):
        with pytest.raises(binding.SprError):
            binding.sched_ops([o])
    s = binding.sched_ops([binding.op(binding.OP_ER, count=2), binding.op(binding.OP_GET_ERROR)])
    assert [o.kind for o in s.ops()] == [binding.OP_ER, binding.OP_GET_ERROR]


def test_mpr_schedule_average_ops():
    binding, _ = _lib()
    K = binding
    ops = binding.sched_mpr(**dict(MPR, G=3)).ops()
    assert [o.kind for o in ops].count(K.OP_AVERAGE) == 1 and ops[-1].kind == K.OP_AVERAGE
    ops = binding.sched_mpr(**dict(MPR, G=3, c_a=0.3)).ops()
    kinds = [o.kind for o in ops]
    assert kinds.count(K.OP_AVERAGE) == 4 and kinds[-1] == K.OP_AVERAGE
    for i, o in enumerate(ops):
        if o.kind == K.OP_CROSSOVER:
            assert ops[i - 1].kind == K.OP_AVERAGE and o.c_a == 0.3
    with pytest.raises(binding.SprError):
        binding.sched_mpr(**dict(MPR, c_a=1.5))


def test_mpr_schedule_monitor_ops():
    binding, _ = _lib()
    K = binding
    ops = binding.sched_mpr(**dict(MPR, G=3, monitor=1)).ops()
    kinds = [o.kind for o in ops]
    mons = [o for o in ops if o.kind == K.OP_MONITOR]
    assert [o.gen for o in mons] == [1, 2, 3]
    for i, o in enumerate(ops):
        if o.kind == K.OP_MONITOR:
            assert ops[i - 1].kind == K.OP_AVERAGE and ops[i - 2].kind == K.OP_SELECT
    assert kinds.count(K.OP_AVERAGE) == 3
    with pytest.raises(binding.SprError):
        binding.sched_ops([binding.op(K.OP_MONITOR, gen=0)])


def test_iteration_trace_flag_validation():
    binding, _ = _lib()
    K = binding
    binding.sched_ops([binding.op(K.OP_RAAR, count=3, beta=0.9, which=K.ITER_TRACE)])
    with pytest.raises(binding.SprError):
        binding.sched_ops([binding.op(K.OP_ER, count=3, which=2)])


def test_header_is_plain_c():
    # the boundary header must compile as C99 on its own (no C++ constructs)
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = "#include <spr.h>\nint main(void) { spr_op o; o.kind = SPR_OP_ER; return o.kind == 0; }\n"
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-fsyntax-only",
                        "-I", inc, "-x", "c", "-"], input=src, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_missing_library_fails_loudly():
    # the product path has no fallback: without the HIP library every call
    # into it raises at load time
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2409_07413_amd import binding\n"
            "binding.LIB_PATH = '/nonexistent/libspr.so'\n"
            "try:\n"
            "    binding.Context(0)\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "    sys.exit(0)\n"
            "sys.exit(1)\n") % ROOT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "not built" in r.stdout


def test_product_code_does_not_use_the_oracle():
    # only the tests, the smoke entry point and the benchmark's CPU baseline
    # may reach the oracle; the package and its native sources never do
    pkg = os.path.join(ROOT, "paper_2409_07413_amd")
    for dirpath, _, files in os.walk(pkg):
        if "_build" in dirpath or "__pycache__" in dirpath:
            continue
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", txt, re.M), f
                assert "oracle/" not in txt and "oracle." not in txt, f


def test_benchmark_reaches_the_oracle_only_in_its_cpu_baseline():
    import ast
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    users = set()
    for fn in ast.walk(tree):
        if isinstance(fn, ast.FunctionDef):
            for node in ast.walk(fn):
                if isinstance(node, ast.ImportFrom) and node.module and node.module.split(".")[0] == "oracle":
                    users.add(fn.name)
                if isinstance(node, ast.Import) and any(a.name.split(".")[0] == "oracle" for a in node.names):
                    users.add(fn.name)
    top = [n for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))
           and "oracle" in ast.dump(n)]
    assert not top
    # cpu_baseline and the workers it runs per member (timing and the
    # device-against-oracle check)
    assert users == {"cpu_baseline", "_oracle_timed", "_oracle_check"}, users


def test_benchmark_finds_its_committed_profiles(monkeypatch):
    # the bench line's `traffic` and `trace_frac` come from the committed
    # rocprofv3 summaries, looked up by kernel name; with the digest the
    # summaries were taken under, every loop kernel the line reports resolves
    import json
    import bench
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic_512_pop64.json")))
    monkeypatch.setattr(bench, "kernel_sources_digest", lambda: t["sources_digest"])
    chunk = t["members_per_launch"]
    for k in ("k_col_proj", "k_row_update_er", "k_row_update_ia"):
        assert bench.measured_traffic(k, chunk) > 0
        assert bench.trace_averages(chunk)[k] > 0
