"""Host logic of the HBM-traffic summary (paper_2403_06654_amd.traffic): the
copy calibration and the per-launch average over the timed kernel classes,
leaving out the dispatches of a gated (queued past the end) Krylov step."""
from paper_2403_06654_amd import traffic


def _row(name, kib):
    return {"Kernel_Name": name, "Counter_Value": str(kib)}


def test_calibration_and_gated_dispatches():
    upd = "void vd::k_gs_update<double, 16>(vd::C2<double>*, ...)"
    row = "void vd::k_row<128, double, 2>(vd::RowArgs, ...)"
    # the 1 GiB copy reads half its bytes by FETCH_SIZE (factor 2), all by WRITE_SIZE
    F = [_row("__amd_rocclr_copyBuffer", 524288), _row(upd, 1000.0), _row(upd, 0.5), _row(upd, 3000.0),
         _row(row, 400.0), _row("void vd::k_mdot<double, 16>(...)", 99.0)]
    W = [_row("__amd_rocclr_copyBuffer", 1048576), _row(upd, 100.0), _row(upd, 0.0), _row(upd, 300.0),
         _row(row, 200.0), _row("void vd::k_mdot<double, 16>(...)", 1.0)]
    out = traffic.summarize(F, W, "abc")
    assert out["csrc_sha256_16"] == "abc"
    assert out["calibration"]["fetch_factor"] == 2.0 and out["calibration"]["write_factor"] == 1.0
    name = "gmres gram-schmidt update (k_gs_update)"
    # the 0.5 KiB dispatch is a gated launch: left out
    assert out["launches"][name] == 2 and out["gated_dispatches_left_out"][name] == 1
    assert out["per_launch_bytes"][name] == round(((1000 + 3000) * 2 + (100 + 300)) * 1024 / 2)
    xname = "pressure x pass (k_row ROW_P)"
    assert out["launches"][xname] == 1 and out["per_launch_bytes"][xname] == (400 * 2 + 200) * 1024


def test_class_patterns_follow_the_grid():
    p5 = traffic.class_patterns(512)
    assert p5["pressure x pass (k_row ROW_P)"].endswith("k_row<256, double, 2>")
    assert p5["pressure z-last (k_col COL_P_LAST)"].endswith("k_col<512, double, 5>")
    import re
    assert re.match(p5["gmres gram-schmidt dots (k_mdot)"], "void vd::k_mdot<double, 16>(x)")
    assert not re.match(p5["gmres gram-schmidt dots (k_mdot)"], "void vd::k_mdot<double, 1>(x)")
