"""Host-side accounting behind the benchmark line (no GPU): the algorithmic bytes per element
and stage of each kernel, written out from the buffer layouts, and the mapping from profiler
kernel names to the bench's kernel keys.

Bytes (FP64, per element and stage, N_s = (p+1)^3 points, N_f = 6 (p+1)^2 face points):
  pre-pass   read U (5 N_s) and the metric terms (10 N_s), write 20 values per face point;
  face       per face point read both sides' 20 values and the face geometry (4), write 10;
             an element owns 3 faces' worth of face points;
  volume     read U, the metric terms and the RK register (20 N_s) and its faces' results
             (10 N_f), write the state and the register (10 N_s): 30 N_s + 10 N_f;
  fused      the volume kernel's bytes plus the pre-pass's writes.
"""
import pytest

import bench
from paper_2308_06605_amd.profiling import short_name


@pytest.mark.parametrize("p", [1, 2, 3, 5, 7])
def test_fp64_bytes_from_layouts(p):
    ns, nfp = (p + 1) ** 3, (p + 1) ** 2
    nf = 6 * nfp
    b = bench.algorithmic_bytes(p, "fp64")
    assert b["prepass"] == 8 * (15 * ns + 20 * nf)
    assert b["face"] == 8 * 3 * nfp * (2 * 20 + 4 + 10)
    assert b["volume"] == 8 * (30 * ns + 10 * nf)
    assert b["volume_pre"] == b["volume"] + 8 * 20 * nf
    # a fused stage (face + fused volume) moves 8 (30 N_s + 57 N_f), a separate one 8 (45 N_s + 57 N_f)
    assert b["face"] + b["volume_pre"] == 8 * (30 * ns + 57 * nf)
    assert b["prepass"] + b["face"] + b["volume"] == 8 * (45 * ns + 57 * nf)
    assert b["stage_min"] == 8 * (45 * ns + 44 * nf)


def test_p3_figures():
    b = bench.algorithmic_bytes(3, "fp64")
    assert (b["prepass"], b["face"], b["volume"], b["volume_pre"]) == (23040, 20736, 23040, 38400)
    assert (b["face"] + b["volume_pre"]) / 64 == 924.0
    assert (b["prepass"] + b["face"] + b["volume"]) / 64 == 1044.0
    assert b["stage_min"] / 64 == 888.0


def test_fp32_fused_bytes():
    p = 3
    nf = 6 * (p + 1) ** 2
    b = bench.algorithmic_bytes(p, "fp32")
    # 20 floats + 3 doubles per face point written by the fused pre-pass
    assert b["volume_pre"] == b["volume"] + (4 * 20 + 8 * 3) * nf
    # the FP32 form's stage minimum: FP64 state (25 N_s doubles), FP32 geometry and face data
    ns = (p + 1) ** 3
    assert b["stage_min"] == 8 * 25 * ns + 4 * (20 * ns + 44 * nf)
    assert b["stage_min"] / ns == 544.0
    assert bench.algorithmic_bytes(7, "fp32")["stage_min"] / 512 == 412.0
    assert bench.algorithmic_bytes(7, "fp64")["stage_min"] / 512 == 624.0


def test_kernel_names():
    assert short_name("void k_volume<3, double, true, false, false, 2, true>(double const*, double*)") == "k_volume_pre"
    assert short_name("void k_volume<3, double, true, false, false, 2, false>(double const*)") == "k_volume"
    assert short_name("void (anonymous namespace)::k_volume32<3, true, 2, true>(double const*)") == "k_volume32_pre"
    assert short_name("void (anonymous namespace)::k_face32<3, true, 256>(float const*)") == "k_face32"
    assert short_name("k_prepass<7, double, true, 1>") == "k_prepass"
    for key in ("prepass", "face", "volume", "volume_pre"):
        assert bench.kernel_name(key, "fp64") == {"prepass": "k_prepass", "face": "k_face", "volume": "k_volume",
                                                  "volume_pre": "k_volume_pre"}[key]
    assert bench.kernel_name("volume_pre", "fp32") == "k_volume32_pre"
    assert bench.kernel_name("prepass", "fp32") == "k_prepass32"


def test_affine_two_pass_minimum():
    """On affine elements the metric terms and face normals are constant per element and face,
    so the two-pass minimum drops them: 8 (25 N_s + 40 N_f), 680 B/DOF at p = 3 and 440 at
    p = 7; the kernels' own bytes are unchanged (they read the per-point terms on every mesh)."""
    a3, c3 = bench.algorithmic_bytes(3, "fp64", affine=True), bench.algorithmic_bytes(3, "fp64")
    assert a3["stage_min"] / 64 == 680.0
    assert bench.algorithmic_bytes(7, "fp64", affine=True)["stage_min"] / 512 == 440.0
    assert {k: v for k, v in a3.items() if k != "stage_min"} == {k: v for k, v in c3.items() if k != "stage_min"}
    assert bench.algorithmic_bytes(3, "fp32", affine=True)["stage_min"] / 64 == 440.0


def test_calibration_copy_is_the_last_copy(tmp_path):
    """The counters are scaled by the run's last device copy (the calibration copy), not by an
    average over every copy that shares its kernel and grid size."""
    from paper_2308_06605_amd.profiling import summarize

    head = ('"Correlation_Id","Dispatch_Id","Agent_Id","Queue_Id","Process_Id","Thread_Id","Grid_Size",'
            '"Kernel_Id","Kernel_Name","Workgroup_Size","LDS_Block_Size","Scratch_Size","VGPR_Count",'
            '"Accum_VGPR_Count","SGPR_Count","Counter_Name","Counter_Value","Start_Timestamp","End_Timestamp"\n')

    def row(d, name, counter, kib):
        return f'{d},{d},"Agent 1",1,1,1,65536,1,"{name}",256,0,0,8,0,16,"{counter}",{kib},0,1\n'

    paths = {}
    for counter, copy_kib, kern_kib in (("FETCH_SIZE", 131072.0, 1000.0), ("WRITE_SIZE", 262144.0, 500.0)):
        p = tmp_path / f"{counter}.csv"
        p.write_text(head + row(1, "__amd_rocclr_copyBuffer", counter, 4 * copy_kib)
                     + row(2, "void k_face<3, double, true, false, false, 256>(int)", counter, kern_kib)
                     + row(3, "__amd_rocclr_copyBuffer", counter, copy_kib))
        paths[counter] = str(p)
    s = summarize(paths["FETCH_SIZE"], paths["WRITE_SIZE"], 256 << 20)
    assert s["fetch_scale"] == pytest.approx(2.0) and s["write_scale"] == pytest.approx(1.0)
    assert s["kernels"]["k_face"]["fetch_bytes"] == pytest.approx(2000.0 * 1024)
    assert s["kernels"]["k_face"]["write_bytes"] == pytest.approx(500.0 * 1024)


def test_stage_line_fused_and_unfused(tmp_path):
    """The stage summary's stage time: face + fused volume kernel with fusion, pre-pass + face +
    volume kernel without (the FP32 p=7 stage the autotuner picks)."""
    import json

    from paper_2308_06605_amd.profiling import algorithmic_bytes, kernel_source_hash, stage_markdown

    stats = tmp_path / "kernel_stats.csv"
    rows = [("void (anonymous namespace)::k_prepass32<7, true, 1>(int)", 0.5),
            ("void (anonymous namespace)::k_face32<7, true, 64>(int)", 0.3),
            ("void (anonymous namespace)::k_volume32<7, true, 1, false>(int)", 0.8),
            ("void (anonymous namespace)::k_volume32<7, true, 1, true>(int)", 1.4)]
    stats.write_text('"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"\n'
                     + "".join(f'"{n}",10,1,{ms * 1e6},1,{ms * 1e6},{ms * 1e6},0\n' for n, ms in rows))
    traffic = tmp_path / "traffic.json"
    traffic.write_text(json.dumps({"kernel_source_hash": kernel_source_hash("fp32"), "prec": "fp32",
                                   "fetch_scale": 2.0, "write_scale": 1.0,
                                   "calibration_copy_bytes": 256 << 20, "kernels": {}, "command": "c"}))
    n, p = 32, 7
    smin = algorithmic_bytes(p, "fp32")["stage_min"] * n ** 3
    for fuse, t in ((False, 0.5 + 0.3 + 0.8), (True, 0.3 + 1.4)):
        text = stage_markdown(str(stats), str(traffic), n, p, "fp32", (1, 2), fuse, "trace")
        line = [l for l in text.splitlines() if l.startswith("Stage (")][0]
        parts = ("k_prepass32 + k_face32 + k_volume32" if not fuse else "k_face32 + k_volume32_pre")
        assert line.startswith(f"Stage ({parts}): {t:.4f} ms"), line
        assert f"{smin / (t * 1e-3) / 8e12:.3f} of 8 TB/s" in line
