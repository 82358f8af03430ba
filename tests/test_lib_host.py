"""Host-side checks of libmgwr (no GPU): exports, validation, and the packed
H-matrix against the independent oracle construction."""
import os
import re
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import workloads as W

mg = pytest.importorskip("paper_1706_07632_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "mgwr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mgwr_[A-Za-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = mg.lib()
    names = _declared_functions()
    assert "mgwr_solve" in names and "mgwr_htrsm" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(mg.EXPORTED)


@pytest.mark.parametrize("kw,msg", [
    (dict(n=64), "2^L - 1"),
    (dict(alpha=1.2), "alpha"),
    (dict(alpha=0.0), "alpha"),
    (dict(M=0), "M must"),
    (dict(k=0), "k must"),
    (dict(k=33), "k must"),
    (dict(dim=3), "dim"),
    (dict(leaf=0), "leaf"),
    (dict(r=0.5), "r >= 1"),
    (dict(nu1=0, nu2=0), "nu1"),
    (dict(gamma=3), "gamma"),
    (dict(precision="mixed", inner_cycles=0), "inner_cycles"),
    (dict(precision="mixed", inner_cycles=17), "inner_cycles"),
    (dict(precision="mixed_bf16", inner_cycles=0), "inner_cycles"),
    (dict(eta=0.0), "eta"),
    (dict(eta=-1.0), "eta"),
    (dict(eta=float("inf")), "eta"),
])
def test_invalid_parameters_are_rejected(kw, msg):
    args = dict(dim=1, n=31, M=64, alpha=0.5, k=8, r=2.0)
    args.update(kw)
    with pytest.raises(mg.MgwrError) as ei:
        mg.Plan(**args)
    assert ei.value.code == mg.MGWR_ERR_INVALID_ARG
    assert msg in str(ei.value)


def test_non_monotone_mesh_rejected():
    t = W.graded_mesh(32, 1.0, 2.0)
    t[5] = t[4]
    with pytest.raises(mg.MgwrError):
        mg.Plan(1, 15, 32, 0.5, k=6, t=t)


CONFIGS = [
    (128, 0.5, 3.0, 8, 16),
    (1024, 0.5, 3.0, 10, 16),
    (512, 0.3, 17 / 3, 10, 16),
    (300, 0.7, 1.857142857142857, 6, 12),
    (100, 0.2, 9.0, 10, 7),
    (33, 0.5, 1.0, 4, 16),
]


@pytest.mark.parametrize("M,alpha,r,k,leaf", CONFIGS)
def test_packed_hmatrix_matches_oracle(M, alpha, r, k, leaf):
    t = W.graded_mesh(M, 1.0, r)
    plan = mg.Plan(1, 15, M, alpha, k=k, t=t, leaf=leaf)
    Rt_lib = plan.export_dense()
    Rt_or = oracle.hmatrix_dense(t, alpha, k, leaf)
    scale = np.max(np.abs(np.diag(Rt_or)))
    assert np.max(np.abs(Rt_lib - Rt_or)) <= 1e-13 * scale
    info = plan.info()
    parts = oracle.block_partition(t, leaf)
    assert info["ndense"] == sum(1 for kind, _, _ in parts if kind == "full")
    assert info["nrk"] == sum(1 for kind, _, _ in parts if kind == "rk")
    tt, a1 = plan.mesh()
    assert np.array_equal(tt, t)
    assert np.max(np.abs(a1 - oracle.initial_value_weights(t, alpha)) / np.abs(a1)) < 1e-13


def test_mesh_formula_when_no_mesh_given():
    plan = mg.Plan(1, 15, 64, 0.4, k=6, r=4.0, T=2.0)
    t, _ = plan.mesh()
    assert np.max(np.abs(t - W.graded_mesh(64, 2.0, 4.0))) <= 4e-16 * 2.0


def test_staging_knobs_and_their_validation():
    plan = mg.Plan(2, 255, 1024, 0.5, k=10, r=3.0)        # levels n = 255 .. 1 (8)
    assert plan.tuned() == {"schedule": "staged", "prefetch": "by_length", "coarse_level": 3}
    plan.set_staging(2, 2)
    assert plan.tuned() == {"schedule": "staged", "prefetch": "deep", "coarse_level": 2}
    plan.set_staging(1, 0)
    assert plan.tuned() == {"schedule": "staged", "prefetch": "shallow", "coarse_level": 0}
    plan.set_staging(0, -1)
    assert plan.tuned()["coarse_level"] == 3 and plan.tuned()["prefetch"] == "by_length"
    for bad in ((3, -1), (-1, -1), (0, 8), (0, -2)):
        with pytest.raises(mg.MgwrError) as ei:
            plan.set_staging(*bad)
        assert ei.value.code == mg.MGWR_ERR_INVALID_ARG
    assert mg.Plan(1, 1023, 512, 0.5, k=8, r=3.0).tuned()["schedule"] == "pipelined"


def test_storage_choice_and_its_validation():
    """2D plans default to colour-split storage, 1D plans are always natural;
    the C entry point rejects unknown values."""
    plan = mg.Plan(2, 31, 64, 0.5, k=6, r=3.0)
    assert plan.info()["layout"] == 1
    plan.set_layout("natural")
    assert plan.info()["layout"] == 0
    plan.set_layout("auto")
    assert plan.info()["layout"] == 1
    with pytest.raises(ValueError):
        plan.set_layout("quincunx")
    for bad in (2, -2, 7):
        assert mg.lib().mgwr_plan_set_layout(plan._h, bad) == mg.MGWR_ERR_INVALID_ARG
    one = mg.Plan(1, 31, 64, 0.5, k=6, r=3.0).set_layout("split")
    assert one.info()["layout"] == 0


def test_bfloat16_factors_take_less_workspace():
    args = (1, 255, 1024, 0.5)
    b64 = mg.Plan(*args, k=10, r=3.0).workspace_bytes()
    b32 = mg.Plan(*args, k=10, r=3.0, precision="mixed").workspace_bytes()
    b16 = mg.Plan(*args, k=10, r=3.0, precision="mixed_bf16").workspace_bytes()
    assert b64 < b16 < b32


def test_workspace_grows_with_grid():
    a = mg.Plan(2, 31, 64, 0.5, k=6, r=3.0).workspace_bytes()
    b = mg.Plan(2, 63, 64, 0.5, k=6, r=3.0).workspace_bytes()
    assert b > 3 * a


@pytest.mark.parametrize("M,alpha,r,k,eta,cluster", [
    (512, 0.5, 3.0, 8, 2.0, "index"), (512, 0.5, 3.0, 8, 0.5, "index"), (1024, 0.3, 17 / 3, 10, 1.0, "geometric"),
    (300, 0.7, 1 / 0.7, 6, 2.0, "geometric"), (256, 0.5, 1.0, 8, 1.0, "geometric"),
])
def test_packed_hmatrix_matches_oracle_for_eta_and_geometric_clusters(M, alpha, r, k, eta, cluster):
    """The general admissibility parameter and the geometric cluster tree in
    the library's host setup against the oracle's independent construction."""
    t = W.graded_mesh(M, 1.0, r)
    plan = mg.Plan(1, 15, M, alpha, k=k, t=t, eta=eta, cluster=cluster)
    Rt_or = oracle.hmatrix_dense(t, alpha, k, 16, eta=eta, cluster=cluster)
    assert np.max(np.abs(plan.export_dense() - Rt_or)) <= 1e-13 * np.max(np.abs(np.diag(Rt_or)))
    parts = oracle.block_partition(t, 16, eta, cluster)
    info = plan.info()
    assert info["ndense"] == sum(1 for kind, _, _ in parts if kind == "full")
    assert info["nrk"] == sum(1 for kind, _, _ in parts if kind == "rk")


def test_unknown_cluster_rule_rejected():
    p = mg.Params()
    mg.lib().mgwr_params_default(mg.ctypes.byref(p))
    p.cluster = 7
    h = mg.ctypes.c_void_p()
    assert mg.lib().mgwr_plan_create(mg.ctypes.byref(p), None, mg.ctypes.byref(h)) == mg.MGWR_ERR_INVALID_ARG
    assert "cluster" in mg.lib().mgwr_last_error().decode()


def _blob(seed=0, layers=(35, 8, 32), rows=None):
    rng = np.random.default_rng(seed)
    n = sum(co * ci * 9 + co for ci, co in zip(layers[:-1], layers[1:]))
    rows = list(range(3, 99, 3)) if rows is None else rows
    return mg.model_blob(layers, 32, rows[:32], 1.0 / 128, rng.standard_normal(n).astype(np.float32)), n


def test_model_blob_is_read_back():
    blob, n = _blob()
    info = mg.describe_model(blob)
    assert info["layers"] == 2 and info["channels"] == [35, 8, 32] and info["nsignal"] == 32
    assert info["nslices"] == 32 and info["rows"][:3] == [3, 6, 9] and info["nparam"] == n
    assert info["h_min"] == 1.0 / 128


def _corrupt(blob, where, value):
    b = bytearray(blob)
    b[where] = value
    return bytes(b)


@pytest.mark.parametrize("case", ["empty", "none", "magic", "version", "truncated", "extra", "checksum",
                                  "nan_weight", "bad_rows", "bad_count"])
def test_missing_or_corrupt_model_is_rejected(case):
    """mgwr_model_describe (host only) returns MGWR_ERR_MODEL for every
    missing or corrupt blob; the same parser guards mgwr_model_load."""
    import struct
    blob, n = _blob()
    header = 8 + 4 + 4 + 3 * 4 + 4 + 4 + 32 * 4 + 8 + 8
    if case == "empty":
        bad = b""
    elif case == "none":
        bad = None
    elif case == "magic":
        bad = _corrupt(blob, 0, ord("X"))
    elif case == "version":
        bad = _corrupt(blob, 8, 2)
    elif case == "truncated":
        bad = blob[:-5]
    elif case == "extra":
        bad = blob + b"\0"
    elif case == "checksum":
        bad = _corrupt(blob, header + 17, blob[header + 17] ^ 1)
    elif case == "nan_weight":
        w = np.frombuffer(blob[header:header + 4 * n], dtype="<f4").copy()
        w[5] = np.nan
        body = blob[:header] + w.tobytes()
        bad = body + struct.pack("<Q", mg._fnv1a64(body))
    elif case == "bad_rows":
        bad, _ = _blob(rows=[5] * 40)
    else:   # parameter count that does not match the shapes
        body = bytearray(blob[:-8])
        struct.pack_into("<q", body, header - 8, n + 1)
        bad = bytes(body) + struct.pack("<Q", mg._fnv1a64(bytes(body)))
    with pytest.raises(mg.MgwrError) as ei:
        mg.describe_model(bad)
    assert ei.value.code == mg.MGWR_ERR_MODEL, case


def test_fnv_checksum_matches_published_vectors():
    """64-bit FNV-1a test vectors (offset basis for the empty string, and "a")."""
    assert mg._fnv1a64(b"") == 0xcbf29ce484222325
    assert mg._fnv1a64(b"a") == 0xaf63dc4c8601ec8c


@pytest.mark.parametrize("args", ["512 0.5 3 8 16 33 2.0 0", "1024 0.3 5.667 10 16 20 1.0 1",
                                  "300 0.7 1.857 6 12 17 2.0 1", "128 0.5 3 8 16 40", "4096 0.5 3 10 16 20", "2048 0.2 9 10 16 16",
                                  "300 0.7 1.857 6 12 17", "100 0.5 1 10 7 16"])
def test_kernel_algorithm_emulated_on_cpu(args):
    """The kernel's per-leaf program (ring of recent leaves, stacked far field,
    accumulator slots, MFMA operand layout) emulated lane by lane on the CPU
    reproduces R~ x and (R~ + c I)^{-1} b of the plan's dense expansion."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "emu")
        subprocess.run([gxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_1706_07632_amd", "csrc"),
                        os.path.join(ROOT, "tests", "native", "march_emu.cpp"),
                        os.path.join(ROOT, "paper_1706_07632_amd", "csrc", "hplan.cpp"), "-o", exe],
                       check=True)
        out = subprocess.run([exe] + args.split(), check=True, capture_output=True, text=True).stdout.split()
    assert float(out[0]) < 1e-12 and float(out[1]) < 1e-12, out


@pytest.mark.parametrize("M,alpha,r,leaf", [(4096, 0.3, 17 / 3, 16), (1024, 0.5, 3.0, 16), (256, 0.5, 1.0, 16),
                                            (300, 0.7, 1 / 0.7, 12)])
def test_near_origin_leaves_flagged_for_float64(M, alpha, r, leaf):
    """Leaves whose steps span more than a factor 8 are the ones float32 cycles
    solve in float64 (graded meshes only; a uniform mesh has none)."""
    plan = mg.Plan(1, 15, M, alpha, k=8, r=r, leaf=leaf)
    t, _ = plan.mesh()
    dt = np.diff(t)
    want = sum(1 for lo in range(0, M, leaf) if dt[lo:lo + leaf].max() > 8.0 * dt[lo:lo + leaf].min())
    assert plan.info()["nf64leaves"] == want
    assert (want > 0) == (r > 1.5)
