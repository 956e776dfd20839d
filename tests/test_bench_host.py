"""Host-side logic of bench.py (no GPU): the one-GPU guard and the counter
traffic it reports only for the kernel source the counters were taken on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def _summary(tmp_path, sha):
    p = tmp_path / "push_kernel_x_pmc.txt"
    p.write_text("# header: not a key\n"
                 "kernel: push_kernel<float>\n"
                 f"kernel_source_sha256_16: {sha}\n"
                 "fetch_bytes_per_launch: 1000\n"
                 "write_bytes_per_launch: 234\n")
    return str(tmp_path / "push_kernel_{}_pmc.txt")


def test_traffic_is_reported_for_the_measured_source_only(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PMC_FILE", _summary(tmp_path, bench.kernel_sha()))
    assert bench.pmc_traffic("x") == 1234.0
    monkeypatch.setattr(bench, "PMC_FILE", _summary(tmp_path, "0" * 16))
    assert bench.pmc_traffic("x") is None
    assert bench.pmc_traffic("missing") is None



def test_benchmark_harris_sheet_follows_the_oracle_relations(orc):
    # the benchmark sets up its double Harris sheet with its own copy of the
    # App. C relations; they must give the oracle's equilibrium (the oracle's
    # relations are pinned to Table 4 and to pressure balance)
    import pic_inputs as W
    cases = [dict(W.HARRIS), dict(W.HARRIS_SMALL),
             dict(W.HARRIS, theta_e=0.1, gu_e=0.40, mass_ratio=1.0),
             dict(W.HARRIS, theta_e=0.3, gu_e=0.5, chi=1.7, mass_ratio=49.0, n_x=7.0)]
    for w in cases:
        hb = bench.harris_parameters(w)
        ho = orc.harris_params(w["theta_e"], w["gu_e"], w["chi"], w["mass_ratio"])
        assert abs(hb["L"] - ho["L_over_de"] * w["n_x"]) < 1e-12 * hb["L"]
        assert abs(hb["b0"] - ho["wce_over_wpe"] / w["n_x"]) < 1e-12 * hb["b0"]
        assert abs(hb["theta_i"] - ho["theta_i"]) < 1e-15
        # the ions drift against the electrons: the oracle gives the signed
        # value, the benchmark the magnitude it loads with the opposite sign
        assert abs(hb["gu_i"] + ho["gu_i"]) < 1e-15
