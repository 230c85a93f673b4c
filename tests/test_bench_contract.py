"""Host-side checks of bench.py: the algorithmic byte model behind its
`GB_s` and `roofline.achieved` figures, and the one-GPU contract."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_byte_model_fp64_and_fp32():
    import bench
    op = bench.pass_bytes_per_voxel(8, 128)
    # pass 1: p and F (2 x 72 B), phase byte, half spectrum (9 x 64/128 x 16 B)
    assert op == {1: 217.0, 2: 144.0, 3: 144.0, 4: 144.0, 5: 144.0}
    assert sum(op.values()) == 793.0
    # x updated every iteration (window 1): pass 1 reads r, p_old, x, F, writes x, p, spectrum
    cg = bench.cg_bytes_per_voxel(8, 128, x_window=1)
    assert cg["pass1"] == 505.0 and cg["pass5"] == 216.0 and sum(cg.values()) == 1153.0
    # window of 8: inside it pass 1 moves 361 B; at its start x and 7 older directions on top
    v = bench.pass1_variant_bytes(8, 128, 8)
    assert v == {"pass1_within_window": 361.0, "pass1_xupdate": 361.0 + 9 * 72}
    cg8 = bench.cg_bytes_per_voxel(8, 128, x_window=8)
    assert cg8["pass1"] == (7 * 361.0 + 361.0 + 9 * 72) / 8 == 442.0 and sum(cg8.values()) == 1090.0
    assert bench.pass1_variant_bytes(8, 128, 1) == {"pass1_within_window": 505.0, "pass1_xupdate": 505.0}
    assert sum(bench.pass_bytes_per_voxel(4, 128).values()) == 397.0
    # odd n2: (n2 + 1) / 2 stored half-line entries
    assert bench.pass_bytes_per_voxel(8, 31)[2] == 2 * 9 * 16 * 16 / 31
    # the 3-kernel lower bound (compulsory I/O + one round trip of the half
    # spectrum with its Nyquist entry per direction): 509.5 B FP64, 255.25 FP32
    assert bench.three_kernel_bytes_per_voxel(8, 128) == 509.5
    assert bench.three_kernel_bytes_per_voxel(4, 128) == 255.25


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0 and "one GPU only" in r.stdout
