"""Host-side logic of bench.py (no GPU): the one-GPU guard and the rule that the HBM byte
count of the main kernel is reported only when its counter summary was taken on the machine code
of the kernel that is timed (a digest of its instructions and its callees', placement aside)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_only_for_the_profiled_kernel_code(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_main_cfg3_eps1e-06_hbm_bytes.txt").write_text(
        "# comment: ignored\nhbm_bytes_per_launch: 1.5e+13\ntile_r: 64\nkernel_code_sha256: abc123\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_code_digest", lambda tile_r: "abc123")
    assert bench.measured_traffic(1e-6, 64) == 1.5e13
    assert bench.measured_traffic(1e-6, 128) is None  # another instantiation was timed
    monkeypatch.setattr(bench, "kernel_code_digest", lambda tile_r: "changed")
    assert bench.measured_traffic(1e-6, 64) is None
    monkeypatch.setattr(bench, "kernel_code_digest", lambda tile_r: None)  # no disassembler
    assert bench.measured_traffic(1e-6, 64) is None
    assert bench.measured_traffic(1e-4, 64) is None  # no summary for this workload


def test_committed_summary_matches_the_built_kernel():
    import pytest
    from paper_2009_12505_amd import build, codeid
    if not os.path.exists(build.LIB) or codeid._objdump() is None:
        pytest.skip("library or disassembler not present")
    assert bench.measured_traffic(1e-6, 64) is not None


def _disasm(base, callee_body):
    """A kernel at ``base`` calling a function placed 0x100 bytes after it."""
    fn = base + 0x100
    off = fn - (base + 8 + 4)  # s_getpc_b64 at base + 8 yields the address of the next instruction
    funcs = {"kern": [(base, "s_load_dwordx2 s[0:1], s[4:5], 0x0"), (base + 4, "s_waitcnt lgkmcnt(0)"),
                      (base + 8, "s_getpc_b64 s[16:17]"),
                      (base + 12, f"s_add_u32 s16, s16, {off & 0xffffffff:#x}"),
                      (base + 20, f"s_addc_u32 s17, s17, {off >> 32}"),
                      (base + 28, "s_swappc_b64 s[30:31], s[16:17]"), (base + 32, "s_endpgm")],
             "fn": [(fn + 4 * i, t) for i, t in enumerate(callee_body)]}
    return funcs, {base: "kern", fn: "fn"}


def test_code_digest_ignores_placement_and_sees_callees():
    from paper_2009_12505_amd import codeid
    body = ["v_add_f64 v[0:1], v[0:1], v[2:3]", "s_setpc_b64 s[30:31]"]
    d1 = codeid.digest_of("kern", *_disasm(0x1000, body))
    d2 = codeid.digest_of("kern", *_disasm(0x5400, body))
    assert d1 == d2  # the same code linked elsewhere
    d3 = codeid.digest_of("kern", *_disasm(0x1000, ["v_mul_f64 v[0:1], v[0:1], v[2:3]", "s_setpc_b64 s[30:31]"]))
    assert d3 != d1  # a changed callee changes the kernel's digest


def test_code_digest_of_the_built_library():
    import pytest
    from paper_2009_12505_amd import build, codeid
    if not os.path.exists(build.LIB) or codeid._objdump() is None:
        pytest.skip("library or disassembler not present")
    d64 = codeid.kernel_code_digest(codeid.k_main_symbol(64, 0))
    assert d64 is not None and len(d64) == 64
    assert codeid.kernel_code_digest(codeid.k_main_symbol(64, 0)) == d64
    assert codeid.kernel_code_digest(codeid.k_main_symbol(64, 1)) != d64
    with pytest.raises(KeyError):
        codeid.kernel_code_digest("_ZN3hfx_no_such_kernel")
