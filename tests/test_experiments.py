"""Host logic of the Sec. 4 experiment runner (no device): which cases each study runs and how
rows are tabulated."""

from paper_2305_04421_amd import experiments as ex
from paper_2305_04421_amd import workloads as wl


def test_weak_series_skips_indivisible_time_step_counts():
    cases = list(ex.weak_cases())
    k80 = sorted({c["nt"] for c in cases if c["steps_per_sub"] == 80})
    assert k80 == [400, 800, 1600, 3200]
    for k in (20, 5):
        assert sorted({c["nt"] for c in cases if c["steps_per_sub"] == k}) == list(ex.NT_SERIES)
    # one- and two-level for every (k, omega, N_t)
    assert len(cases) == 2 * 3 * (4 + 6 + 6)
    assert all(c["mesh"] == 17 for c in cases)


def test_cases_are_valid_problems():
    from paper_2305_04421_amd import _lib
    import ctypes
    lib = _lib.load()
    for c in list(ex.weak_cases()) + list(ex.omega_cases()) + list(ex.mesh_cases()):
        params = wl.paper_problem(c["nt"], c["steps_per_sub"], c["omega"], coarse=c["coarse"],
                                  n_points=c["mesh"])
        assert params["n_sub"] * c["steps_per_sub"] == c["nt"]
        prob = _lib.make_problem(params, "fp64", "step")
        assert lib.kkt_validate(ctypes.byref(prob)) == 0, c


def test_markdown_marks_unconverged_runs():
    rows = [dict(study="weak", mesh=17, steps_per_sub=20, omega=1e-2, coarse=c, nt=nt,
                 iters=it, converged=conv)
            for c, nt, it, conv in [(0, 100, 22, True), (0, 200, 420, False),
                                    (2, 100, 20, True), (2, 200, 21, True)]]
    text = ex.markdown(rows)
    lines = text.splitlines()
    assert lines[0].startswith("| mesh | steps/sub | omega | level | N_t=100 | N_t=200 |")
    assert "| 17 | 20 | 0.01 | one-level | 22 | >420 |" in lines
    assert "| 17 | 20 | 0.01 | two-level | 20 | 21 |" in lines


def test_ablation_cases_are_valid_problems_on_the_modal_path():
    from paper_2305_04421_amd import _lib
    import ctypes
    lib = _lib.load()
    cases = list(ex.ablation_cases())
    assert {c["variant"] for c in cases} == set(ex.ABLATIONS)
    for c in cases:
        params = wl.paper_problem(c["nt"], c["steps_per_sub"], c["omega"], coarse=c["coarse"],
                                  n_points=c["mesh"])
        params.update(ex.ABLATIONS[c["variant"]])
        prob = _lib.make_problem(params, "fp64", "modal")
        assert lib.kkt_validate(ctypes.byref(prob)) == 0, c


def test_ablation_table_lists_variants_in_order():
    rows = [dict(study="ablation", variant=v, mesh=17, steps_per_sub=5, omega=1e-2, coarse=2, nt=nt,
                 iters=10 + i, converged=True)
            for i, v in enumerate(["ASM", "paper"]) for nt in (100, 200)]
    lines = ex.markdown(rows).splitlines()
    assert lines[0] == "| steps/sub | omega | variant | N_t=100 | N_t=200 |"
    assert lines[2].startswith("| 5 | 0.01 | paper | 11 | 11 |")
    assert lines[3].startswith("| 5 | 0.01 | ASM | 10 | 10 |")


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
