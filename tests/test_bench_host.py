"""Host-side pieces of the benchmark: the CPU oracle baseline's timing split
and the host record (no GPU)."""
import numpy as np


def test_cpu_baseline_splits_factorisation_from_solves():
    import bench
    from oracle.hdg import HdgOracle
    import hdg_inputs as hi

    out, (ns, r, q, lam) = bench.cpu_baseline(16, 1, 0.5, repeats=2)
    assert ns == 8 and out["kind"] == "oracle" and out["cores"] == 1
    scale = (16 / 8) ** 2
    assert np.isclose(out["value"], 1.0 / (out["solve_s"] * scale), rtol=1e-3)
    assert out["value_incl_factor"] < out["value"]
    assert all(b["threads"] == 1 for b in out["host"]["blas"])
    assert out["host"]["cpu_count"] >= out["host"]["affinity"] >= 1
    # the split steps give the oracle's own one-call solution
    q_ref, lam_ref = HdgOracle(hi.torus(8), 1, 0.5, 1.0, 1.0, 1.0).solve(r)
    assert np.allclose(lam, lam_ref, rtol=0, atol=1e-12 * np.abs(lam_ref).max())
    assert np.allclose(q, q_ref, rtol=0, atol=1e-12 * np.abs(q_ref).max())


def test_oracle_per_config_reports_every_workload(monkeypatch):
    import bench
    import hdg_inputs as hi

    # a level-2 sphere keeps the test short; the record's shape is what is checked
    real = hi.icosphere_hierarchy
    monkeypatch.setattr(hi, "icosphere_hierarchy", lambda level, *a, **k: real(2, *a, level_coarse=0))
    out = bench.oracle_per_config(repeats=1)
    assert set(out) == {"torus8x8_p1_courant4", "icosphere_L6_p2_dt1800", "icosphere_L7_p3_dt3600"}
    for rec in out.values():
        assert rec["value"] > 0 and rec["cores"] == 1 and rec["factor_s"] >= 0
    assert out["torus8x8_p1_courant4"]["sample"] == "full size"
    assert out["torus8x8_p1_courant4"]["trace_unknowns"] == 192 * 2
