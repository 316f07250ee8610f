"""Host-side parts of the benchmark: the one-GPU refusal, the convolution work
counts and the parsing of the committed profiler summaries (no GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_convolution_counts_follow_the_layer_shapes():
    import bench
    fl, by = bench.conv_counts(1)
    # forward: 2 x out pixels x Cout x 9 Cin per layer of the 128 x 128 network
    layers = [(128 * 128, 32, 2), (64 * 64, 32, 32), (32 * 32, 32, 32), (32 * 32, 1, 32)]
    fwd = sum(2 * px * co * 9 * ci for px, co, ci in layers)
    assert fl["conv_fwd"] == fwd == 113_836_032
    assert fl["conv_bwd_weight"] == fwd
    assert fl["conv_bwd_data"] == fwd - layers[0][0] * 2 * 32 * 9 * 2   # no input gradient of layer 1
    # forward bytes: BF16 inputs and outputs, FP32 network output
    assert by["conv_fwd"] == ((2 * 128 * 128 * 2 + 2 * 128 * 128 * 32) +     # layer 1 in, out
                              (2 * 128 * 128 * 32 + 2 * 64 * 64 * 32) +     # layer 2 (stride 2)
                              (2 * 64 * 64 * 32 + 2 * 32 * 32 * 32) +       # layer 3 (stride 2)
                              (2 * 32 * 32 * 32 + 4 * 32 * 32))             # layer 4, FP32 out
    fl8, by8 = bench.conv_counts(8)
    assert all(abs(fl8[k] - 8 * fl[k]) < 1e-6 * fl8[k] for k in fl)


def test_committed_profiles_parse():
    from paper_2608_06853_amd import profsummary
    tr = profsummary.read_traffic(os.path.join(ROOT, "profiles", "c2_clinical_hbm_traffic.txt"))
    co = profsummary.read_counters(os.path.join(ROOT, "profiles", "c2_clinical_valu_counters.txt"))
    for fam in ("path_adj", "table", "das_fwd", "das_adj", "cmpe"):
        assert tr[fam][1] > 0 and len(tr[fam][0]) == 16
        assert co[fam][1] > 0 and 0 < co[fam][2] <= 1
