"""The benchmark's byte models, kernel naming and profile lookups (CPU only)."""
import hashlib
import os

import bench


def test_field_and_pass_bytes():
    R, C = bench.field_bytes(512)
    assert R == 4 * 512 ** 3 and C == 8 * 512 * 512 * 257
    pb = bench.pass_bytes(512)
    assert pb["z_r2c"] == pb["z_c2r"] == R + C
    assert pb["y_fwd"] == pb["x_inv"] == 2 * C
    # the pair's pass traffic: 2R + 10C
    assert sum(pb.values()) == 2 * R + 10 * C


def test_solver_pass_bytes_match_the_transit_layout():
    """K = 170 kept modes per axis at 512^3, transit rows of 176 complex values: P2 reads
    the 6 fields' kept ky rows and writes all 512 (1475.0 / 2214.6 MB)."""
    pb = bench.ns_pass_bytes(512)
    K, KZP = 170, 176
    assert pb["P2"] == (6 * 512 * KZP * (2 * K + 1) * 8, 6 * 512 * KZP * 512 * 8)
    assert round(pb["P2"][0] / 1e6, 1) == 1475.0 and round(pb["P2"][1] / 1e6, 1) == 2214.6
    assert pb["P5+P1"] == (pb["P5"][0] + pb["P5"][1], pb["P5"][1] + pb["P1"][1])


def test_kernel_names_from_plan_descriptions():
    desc = {0: "z N=512 LPW=16 E=8 nt=512 lds=38016",
            1: "y L=512 W=16 E=16 v=2 nt=512 lds=73728",
            2: "x L=512 W=16 E=8 v=0 nt=1024 lds=73728"}
    names = bench.kernel_names(desc, 512)
    assert names["z_r2c"] == "k_z_r2c<float, 256, 8, 16>"
    assert names["y_fwd"] == names["y_inv"] == "k_strided_pp<float, 512, 16, 16, false, 1>"
    assert names["x_fwd"] == "k_strided<float, 512, 8, 16, false, false>"
    desc[1] = "y L=512 W=16 E=16 v=8 nt=512 lds=73728"   # two workgroups per CU: 4 waves per SIMD
    assert bench.kernel_names(desc, 512)["y_fwd"] == "k_strided_pp<float, 512, 16, 16, false, 4>"
    desc[2] = "x L=1024 W=16 E=32 v=6 nt=512 lds=77824"  # split exchanges
    assert bench.kernel_names(desc, 1024)["x_fwd"] == "k_strided<float, 1024, 32, 16, false, true>"


def test_profile_record_checks_the_source_digest(tmp_path):
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = b""
    for f in ("fft_core.hpp", "fft_kernels.hpp"):
        with open(os.path.join(here, "paper_1805_07801_amd", "csrc", f), "rb") as fh:
            src += fh.read()
    digest = hashlib.sha256(src).hexdigest()[:16]
    p = tmp_path / "summary.txt"
    p.write_text("# a summary\nsource_digest %s x\ntraffic_bytes_per_launch k_a<float,8> 123\n" % digest)
    args = (str(p), ("fft_core.hpp", "fft_kernels.hpp"), "traffic_bytes_per_launch")
    assert bench.profile_record(*args, "k_a<float, 8>") == 123.0
    assert bench.profile_record(*args, "k_b<float, 8>") is None
    p.write_text("source_digest 0000000000000000 x\ntraffic_bytes_per_launch k_a<float,8> 123\n")
    assert bench.profile_record(*args, "k_a<float, 8>") is None  # sources changed since


def test_p3_kernel_name_follows_the_tile_cache():
    assert bench.p3_kernel_name(512).startswith("k_ns_p3<float, 256, ")
