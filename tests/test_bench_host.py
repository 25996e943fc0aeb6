"""Host-side logic of bench.py (no GPU): the one-GPU contract, the traffic
profile's keying on the kernel sources and launch configuration, and the
algorithmic byte counts it prices the loops with."""
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEFAULT_KEY = ("n=160 variant=owner renumber=morton cluster=512 block=512 lane_groups=True "
               "colour_sort=False bank_spread=True halo_order=True")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_profile_applies_only_to_its_sources_and_configuration():
    # the committed counter summary names the sources' hash and the configuration
    kv = {}
    with open(bench.TRAFFIC_PROFILE) as f:
        for ln in f:
            if ":" in ln and not ln.startswith("#"):
                k, v = ln.split(":", 1)
                kv[k.strip()] = v.strip()
    t = bench.measured_traffic(kv["config"])
    if kv["sources_sha256"] == bench.sources_sha():
        assert t == float(kv["traffic_bytes_per_launch"])
        assert 1.0 < t / float(kv["algorithmic_bytes_per_launch"]) < 2.0
    else:
        assert t is None  # kernels changed since the counters were taken
    assert bench.measured_traffic(DEFAULT_KEY.replace("bank_spread=True", "bank_spread=False")) is None
    assert bench.measured_traffic(DEFAULT_KEY.replace("n=160", "n=100")) is None


def test_algorithmic_bytes():
    E, N = 26624000, 4096000
    per = lambda k: bench.BYTES[k][0] * E + bench.BYTES[k][1] * N
    assert per("fp64") == 1245184000          # map 8 + n 24; q 48 + res 48
    assert per("fp32") == 827392000           # map 8 + n 12; q 24 + res 48
    assert per("adjoint") == 2080768000       # + nbar 24; q, rbar, qbar 48 each
    assert per("fp64_fused") == 1474560000    # q 48 + q0 48 + vol 8 + q 48
    assert bench.BYTES["rk64"] == (0, 152) and bench.BYTES["rk32"] == (0, 104)
    # the FP32-storage loop moves 1/1.505 of the FP64 loop's bytes
    assert abs(per("fp64") / per("fp32") - 1.505) < 1e-3


def test_cpu_baseline_reports_gpu_errors_against_the_oracle():
    # the oracle leg compares residuals handed to it with its own: an exact copy
    # scores 0, a copy with one value off by 1e-6 of its variable's largest
    # magnitude scores 1e-6
    import meshgen
    import oracle
    m = meshgen.build_mesh(4, 0, 0.1)
    q = meshgen.state(m.N, m.perm)
    ref = oracle.residual(m.e2n, q, m.w)
    off = ref.copy()
    off[2, 5] += 1e-6 * np.abs(ref[2]).max()
    cb = bench.cpu_baseline(m, q, {"same": ref, "off": off}, seconds=0.01)
    assert cb["kind"] == "oracle" and cb["value"] > 0
    assert cb["gpu_residual_error_vs_oracle"]["same"] == 0.0
    assert abs(cb["gpu_residual_error_vs_oracle"]["off"] - 1e-6) < 1e-9
