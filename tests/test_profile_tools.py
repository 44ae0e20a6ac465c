"""Host-side tools behind the reported roofline numbers (CPU only): the counter
summary that turns FETCH_SIZE / WRITE_SIZE readings into bytes per launch, the
lookup of committed traffic records, and the kernel names the benchmark
reports for a launch shape."""
import csv
import json

import profile_run as pr

FIELDS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
STRIPS = {"groups_per_cu": 2, "ilp": 1, "streaming": 0, "compact": 1, "tiled": 5, "steps": 8}


def _counters(d, rows):
    d.mkdir()
    with open(d / "c_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, grid, value) in enumerate(rows):
            w.writerow(dict(Dispatch_Id=i + 1, Kernel_Name=name, Grid_Size=grid,
                            Counter_Name="X", Counter_Value=value))


def test_summary_calibrates_on_the_large_copies_only(tmp_path):
    """A workload's own one-state copies (here 64 MiB) must not enter the
    calibration by the 512 MiB copies, even with the same grid size."""
    kern = "void kpm::k_moment_march_re<HIP_vector_type<double, 2u>, true, 8>(kpm::Ell)"
    other = "void kpm::k_moment_march<HIP_vector_type<double, 2u>, true, false, 8>(kpm::Ell)"
    copy = "__amd_rocclr_copyBuffer"
    # counters read half the true KiB for copies (a factor 2 to recover)
    tail = "void kpm::k_moment_march_re<HIP_vector_type<double, 2u>, true, 5>(kpm::Ell)"
    # another kernel and a shorter pass of the same kernel (a moment set's
    # tail) stay out of the launch's average
    fetch = [(copy, 512, 32768.0), (kern, 1024, 1000.0), (kern, 1024, 1200.0),
             (other, 1024, 9999.0), (tail, 1024, 7777.0)] + [(copy, 512, 262144.0)] * 3
    write = [(copy, 512, 65536.0), (kern, 1024, 500.0), (kern, 1024, 500.0)] + \
            [(copy, 512, 524288.0)] * 3
    _counters(tmp_path / "f", fetch)
    _counters(tmp_path / "w", write)
    meta = dict(kernel="k_moment_march_re<double2,true,8> (fp64, 1 vector(s))", kernel_sha="abc",
                step_rows=100, launch_shape=STRIPS, copy_mib=512, step_bytes=2_000_000,
                command="cmd")
    (tmp_path / "meta.json").write_text(json.dumps(meta))
    out = tmp_path / "t.json"
    pr.summarize(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "meta.json"), str(out))
    r = json.loads(out.read_text())
    assert r["fetch_kib_per_launch"] == 1100.0 and r["write_kib_per_launch"] == 500.0
    assert r["fetch_scale"] == 2.0 and r["write_scale"] == 1.0
    assert r["bytes_per_launch"] == (1100 * 2 + 500) * 1024
    assert r["traffic_over_algorithmic"] == round((1100 * 2 + 500) * 1024 / 2_000_000, 4)


def test_traffic_lookup_matches_version_size_shape_and_name(tmp_path):
    sha = pr.kernel_sha(STRIPS)
    recs = [dict(kernel="k_moment_march<double2,true,false,8> (fp64, 1 vector(s))",
                 kernel_sha=sha, step_rows=100, launch_shape=STRIPS, bytes_per_launch=111),
            dict(kernel="k_moment_march_re<double2,true,8> (fp64, 1 vector(s))",
                 kernel_sha=sha, step_rows=100, launch_shape=STRIPS, bytes_per_launch=222)]
    p = tmp_path / "r.json"
    p.write_text(json.dumps({"records": recs}))
    assert pr.measured_traffic(str(p), 100, STRIPS) == 111
    assert pr.measured_traffic(str(p), 100, STRIPS, "k_moment_march_re<double2,true,8>") == 222
    assert pr.measured_traffic(str(p), 101, STRIPS) is None
    assert pr.measured_traffic(str(p), 100, dict(STRIPS, steps=7)) is None
    stale = dict(recs[0], kernel_sha="0" * 16)
    p.write_text(json.dumps({"records": [stale]}))
    assert pr.measured_traffic(str(p), 100, STRIPS) is None


def test_reported_kernel_names():
    assert pr.moment_kernel_name("double2", STRIPS, False) == "k_moment_march<double2,true,false,8>"
    assert pr.moment_kernel_name("double2", STRIPS, True) == "k_moment_march<double2,true,true,8>"
    assert pr.moment_kernel_name("double2", STRIPS, False, real=True) == \
        "k_moment_march_re<double2,true,8>"
    # the doubling form has no real-part variant; several vectors take single steps
    assert pr.moment_kernel_name("double2", STRIPS, True, real=True) == \
        "k_moment_march<double2,true,true,8>"
    assert pr.moment_kernel_name("float2", STRIPS, False, n_vec=64).startswith("k_moment_step<")
    tiles = dict(STRIPS, tiled=2, steps=4)
    assert pr.moment_kernel_name("double2", tiles, False, real=True) == \
        "k_moment_stepk<double2,true,false,4,4>"


def test_joint_shape():
    """The two-plane shape of the joint VAC / MSD call: the one-vector grid's
    wavefronts over both planes in groups of 256 threads, ten steps per pass
    where the one-vector FP64 strips take eight."""
    j = pr.joint_shape(STRIPS, 256)
    assert j == dict(STRIPS, steps=10, vectors_per_wave=1, plane_groups=256)
    small = dict(STRIPS, groups_per_cu=8, group_size=64)
    assert pr.joint_shape(small, 256) == dict(STRIPS, groups_per_cu=8, steps=10,
                                              vectors_per_wave=1, plane_groups=256)
    assert pr.joint_shape(STRIPS, 256, fp64=False)["steps"] == 8
    assert pr.joint_shape(dict(STRIPS, steps=6), 256)["steps"] == 6
    assert pr.moment_kernel_name("double2", j, False, 2, real=True, onsf=False) == \
        "k_moment_march_re<double2,false,10>"


def test_real_part_sets_of_several_vectors():
    """Real-part sets of several vectors kept vector-major run ten steps per
    pass with FP64 states, eight in the FP32 forms."""
    planar = dict(STRIPS, vectors_per_wave=1, plane_groups=16)
    assert pr.re_launch(planar, "fp64", 64)["steps"] == 10
    assert pr.re_launch(planar, "fp32_arith", 64)["steps"] == 8
    assert pr.re_launch(planar, "fp32", 64)["steps"] == 8
    assert pr.re_launch(planar, "fp64", 1)["steps"] == 8
    assert pr.re_launch(dict(planar, group_size=64), "fp64", 64)["steps"] == 8
    assert pr.moment_kernel_name("double2", pr.re_launch(planar, "fp64", 64), False, 64,
                                 real=True, onsf=False) == "k_moment_march_re<double2,false,10>"
