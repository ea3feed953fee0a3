"""The C-ABI library loads, exports every symbol the header declares, and
validates its descriptors on the host -- no GPU compute calls."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(restore_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def R():
    from paper_2409_07148_amd import restore
    return restore


def test_library_exports_every_declared_symbol(R):
    declared = _declared_functions()
    assert "restore_init" in declared and "restore_step" in declared and "restore_estimate" in declared
    out = subprocess.run(["nm", "-D", "--defined-only", R.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (restore_[a-z_0-9]+)$", out, flags=re.M))
    missing = [n for n in declared if n not in exported]
    assert not missing, missing
    for n in declared:
        assert hasattr(R._lib, n)


def test_binding_names_match_header(R):
    for n in _declared_functions():
        assert callable(getattr(R, n)), n


def _problem(R, **kw):
    from workloads import gmm_full
    return R.problem_from_workload(gmm_full(n_chains=1000), **kw)


def test_state_bytes_grows_with_chains(R):
    p1 = _problem(R)
    b1 = R.restore_state_bytes(p1.target, p1.mu, p1.local, p1.cfg)
    p2 = _problem(R, n_chains=4000)
    b2 = R.restore_state_bytes(p2.target, p2.mu, p2.local, p2.cfg)
    assert b2 > b1 > 0
    # per chain: x, grad (8 floats each), 2 doubles and 8 further words
    assert b2 - b1 >= 3000 * (16 * 4 + 16 + 8 * 4)


@pytest.mark.parametrize("field,value,status", [
    ("c_tilde", -1.0, -1), ("n_chains", 0, -1), ("drain_cap", -3, -1), ("block_size", 96, -1),
    ("first_chain", -1, -1),
])
def test_config_validation(R, field, value, status):
    p = _problem(R)
    setattr(p.cfg, field, value)
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert e.value.status == status
    assert R.restore_last_error()


def test_target_validation(R):
    p = _problem(R)
    p.target.dim = 0
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert e.value.status == R.E_INVALID_ARG
    p = _problem(R)
    p.target.params_count -= 1
    with pytest.raises(R.RestoreError):
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    p = _problem(R)
    p._params[5] = np.nan
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert e.value.status == R.E_NONFINITE


def test_local_kernel_validation(R):
    # large steps belong to the MH chain (c_tilde = 0); restore runs M^0
    p = _problem(R)
    p.local.large_step_prob = 0.3
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert e.value.status == R.E_UNSUPPORTED
    p.cfg.c_tilde = 0.0
    assert R.restore_state_bytes(p.target, p.mu, p.local, p.cfg) > 0
    p.local.large_step_prob = 1.5
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert e.value.status == R.E_INVALID_ARG
    # HMC needs 1..64 leapfrog steps; the other kernels take none
    for kind, n, ok in ((R.LOCAL_HMC, 8, True), (R.LOCAL_HMC, 0, False), (R.LOCAL_HMC, 65, False),
                        (R.LOCAL_MALA, 1, False)):
        p = _problem(R)
        p.local.kind, p.local.n_leapfrog = kind, n
        if ok:
            assert R.restore_state_bytes(p.target, p.mu, p.local, p.cfg) > 0
        else:
            with pytest.raises(R.RestoreError) as e:
                R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
            assert e.value.status == R.E_INVALID_ARG
    p = _problem(R)
    p.local.step = 0.0   # MALA needs a positive step
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert e.value.status == R.E_INVALID_ARG


def test_unadjusted_jump_process_validation(R):
    """The unadjusted random-walk jump process (not pi-invariant, general
    killing rate) is built for the isotropic mixture with the uniform mu
    and needs c_tilde > 0 and a positive jump size; its slab carries the
    Q^T p terms (4 floats per component more)."""
    from workloads import gmm_iso_2d, gmm_iso_2d_unadjusted
    wl = gmm_iso_2d_unadjusted(n_chains=1000)
    p = R.problem_from_workload(wl)
    assert p.local.kind == R.LOCAL_RW_UNADJUSTED
    n_rwu = R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    q = R.problem_from_workload(gmm_iso_2d(n_chains=1000))
    assert n_rwu >= R.restore_state_bytes(q.target, q.mu, q.local, q.cfg) > 0
    p = R.problem_from_workload(wl)
    p.cfg.c_tilde = 0.0
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert e.value.status == R.E_INVALID_ARG
    p = R.problem_from_workload(wl)
    p.local.step = 0.0
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert e.value.status == R.E_INVALID_ARG
    p = _problem(R)   # full-covariance target: no closed-form Q^T p
    p.local.kind = R.LOCAL_RW_UNADJUSTED
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert e.value.status == R.E_UNSUPPORTED


def test_init_rejects_null_and_small_buffers(R):
    p = _problem(R)
    n = R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    with pytest.raises(R.RestoreError) as e:
        R.restore_init(p.target, p.mu, p.local, p.cfg, 0, n, stream=0)
    assert e.value.status == R.E_INVALID_ARG
    with pytest.raises(R.RestoreError) as e:
        R.restore_init(p.target, p.mu, p.local, p.cfg, 256, n - 1, stream=0)
    assert e.value.status == R.E_BUFFER_TOO_SMALL
    with pytest.raises(R.RestoreError) as e:
        R.restore_init(p.target, p.mu, p.local, p.cfg, 256 + 4, n, stream=0)
    assert e.value.status == R.E_INVALID_ARG


def _pss_problem(R, **kw):
    from workloads import pss_render
    return R.problem_from_workload(pss_render(n_chains=1000, image=(64, 64)), **kw)


@pytest.mark.parametrize("batches,status", [(-1, -1), (4097, -1), (1001, -1)])
def test_image_batches_validation(R, batches, status):
    p = _pss_problem(R)
    p.cfg.image_batches = batches
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert e.value.status == status


def test_image_batches_need_the_pixel_integrand(R):
    p = _problem(R)
    p.cfg.image_batches = 4
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert e.value.status == R.E_INVALID_ARG


def test_image_pixel_index_stays_in_int32(R):
    p = _pss_problem(R, n_chains=100000)
    p.cfg.image_w, p.cfg.image_h, p.cfg.image_batches = 16384, 16384, 16
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert e.value.status == R.E_INVALID_ARG


def test_splat_binning_sizes_the_state(R):
    """Binned splats hold buckets for 1.5 x one 64-step launch of records
    (8 bytes each) plus the partial tiles; the direct path needs none."""
    binned = _pss_problem(R, n_chains=8192)
    direct = _pss_problem(R, n_chains=8192, flags=R.FLAG_SPLAT_DIRECT)
    nb = R.restore_state_bytes(binned.target, binned.mu, binned.local, binned.cfg)
    nd = R.restore_state_bytes(direct.target, direct.mu, direct.local, direct.cfg)
    records = 8192 * 65
    assert nb - nd >= 1.5 * records * 8
    assert nb - nd <= 1.5 * records * 8 + 16 * 16 * 65536 + 65536 + 16 * 4096


def test_nll_and_mlp_argument_validation(R):
    shape = R.restore_mlp_shape(12, 64, 65, 8)
    with pytest.raises(R.RestoreError) as e:
        R.restore_mlp_param_count(shape)
    assert e.value.status == R.E_INVALID_ARG
    n, a = R.restore_mlp_param_count(R.restore_mlp_shape(12, 64, 64, 8))
    assert n == 64 * 12 + 64 + 64 * 64 + 64 + 1088 * 64 + 1088 and a == 4 * 64
    # precision: AUTO, FP32 (widths up to 256) or BF16
    for p, status in ((3, R.E_INVALID_ARG), (-1, R.E_INVALID_ARG)):
        with pytest.raises(R.RestoreError) as e:
            R.restore_mlp_param_count(R.restore_mlp_shape(12, 64, 64, 8, p))
        assert e.value.status == status
    with pytest.raises(R.RestoreError) as e:
        R.restore_mlp_param_count(R.restore_mlp_shape(12, 257, 64, 8, R.MLP_FP32))
    assert e.value.status == R.E_UNSUPPORTED
    assert R.restore_mlp_param_count(R.restore_mlp_shape(12, 257, 64, 8, R.MLP_BF16))[0] > 0
    assert R.restore_mlp_param_count(R.restore_mlp_shape(12, 257, 64, 8, R.MLP_AUTO))[0] > 0
    # partial sums of up to 256 workgroups and the totals, 34 rows of 64 (d = 16),
    # and one line for the completion counter of the sum launch
    assert R.restore_gmm_nll_workspace_bytes() == 257 * 34 * 64 * 8 + 64 * 8
    with pytest.raises(R.RestoreError) as e:
        R.restore_adam_step(0, 0, 0, 0, 10, 1, 1e-3, stream=0)
    assert e.value.status == R.E_INVALID_ARG


def test_reset_sums_rejects_null_context(R):
    with pytest.raises(R.RestoreError) as e:
        R.restore_reset_sums(None, stream=0)
    assert e.value.status == R.E_INVALID_ARG


def test_batch_rejects_the_mh_chain(R):
    """Batched targets are restore problems; c_tilde = 0 (the MH chain)
    runs on the single-target path."""
    from workloads import gmm_full
    wl = gmm_full(n_chains=1000)
    p = R.make_problem("gmm_full", wl.d, wl.K, wl.params, local="rwmh", step=0.02, n_chains=1000,
                       c_tilde=1.0, seed=1, drain_cap=64)
    assert R.restore_batch_state_bytes([p.target], [p.local], [p.cfg]) > 0
    p.cfg.c_tilde = 0.0
    with pytest.raises(R.RestoreError) as e:
        R.restore_batch_state_bytes([p.target], [p.local], [p.cfg])
    assert e.value.status == R.E_UNSUPPORTED


def test_batch_mu_descriptors(R):
    """A learned-form mu adds its slab to the batch state; invalid entries
    are rejected on the host."""
    from workloads import gmm_full
    wl = gmm_full(n_chains=1000)
    p = R.make_problem("gmm_full", wl.d, wl.K, wl.params, local="rwmh", step=0.02, n_chains=1000,
                       c_tilde=1.0, seed=1, drain_cap=64)
    base = R.restore_batch_state_bytes([p.target], [p.local], [p.cfg])
    uni = R.restore_mu(R.MU_UNIFORM_BOX, 0, 0.0, 0, None)
    assert R.restore_batch_state_bytes([p.target], [p.local], [p.cfg], [uni]) == base
    # the device row is only read by restore_batch_init: any non-null address sizes the state
    gmm = R.restore_mu(R.MU_GMM_DIAG, 64, 0.1, 0, 256)
    assert R.restore_batch_state_bytes([p.target], [p.local], [p.cfg], [gmm]) > base
    for bad in (R.restore_mu(R.MU_GMM_DIAG, 0, 0.1, 0, 256), R.restore_mu(R.MU_GMM_DIAG, 8, 1.5, 0, 256),
                R.restore_mu(R.MU_GMM_DIAG, 8, 0.1, 0, None), R.restore_mu(7, 8, 0.1, 0, 256)):
        with pytest.raises(R.RestoreError) as e:
            R.restore_batch_state_bytes([p.target], [p.local], [p.cfg], [bad])
        assert e.value.status == R.E_INVALID_ARG


def test_tile_stratified_validation(R):
    """Tiles need the pixel integrand, the uniform mu, c_tilde > 0, an edge
    of 1..64 pixels and max(1, image_batches) chains per tile; they shrink
    the state (no splat buckets)."""
    p = _pss_problem(R)
    binned = R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    p.cfg.tile_px = 64
    tiled = R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert 0 < tiled < binned
    # 16 tiles of 16 x 16 on the 64 x 64 image: 62 or 63 chains per tile
    for field, value, status in (("tile_px", 65, R.E_INVALID_ARG), ("tile_px", -1, R.E_INVALID_ARG),
                                 ("c_tilde", 0.0, R.E_UNSUPPORTED), ("image_batches", 63, R.E_INVALID_ARG)):
        q = _pss_problem(R)
        q.cfg.tile_px = 16
        setattr(q.cfg, field, value)
        with pytest.raises(R.RestoreError) as e:
            R.restore_state_bytes(q.target, q.mu, q.local, q.cfg)
        assert e.value.status == status, (field, value)
    q = _pss_problem(R)
    q.cfg.tile_px = 16
    q.cfg.integrands &= ~R.INTEGRAND_PIXEL
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(q.target, q.mu, q.local, q.cfg)
    assert e.value.status == R.E_INVALID_ARG
    # the chain-to-tile map spans the whole population: no chain offset
    q = _pss_problem(R)
    q.cfg.tile_px = 16
    q.cfg.first_chain = 1000
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(q.target, q.mu, q.local, q.cfg)
    assert e.value.status == R.E_UNSUPPORTED
    q = _pss_problem(R)
    q.cfg.tile_px = 16
    q.mu = R.restore_mu(R.MU_GMM_DIAG, 8, 0.1, 0, 256)
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(q.target, q.mu, q.local, q.cfg)
    assert e.value.status == R.E_UNSUPPORTED


def test_binding_refuses_to_load_without_the_library(tmp_path):
    """No fallback: a copy of the binding next to no library raises
    ImportError on import (the product path never runs without the HIP
    kernels)."""
    import shutil
    import sys
    pkg = tmp_path / "pkg_copy"
    pkg.mkdir()
    here = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2409_07148_amd")
    shutil.copy(os.path.join(here, "restore.py"), pkg / "restore.py")
    (pkg / "__init__.py").write_text("")
    r = subprocess.run([sys.executable, "-c", "import pkg_copy.restore"], cwd=tmp_path, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "no fallback" in r.stderr


def test_fixed_point_image_flag(R):
    """RESTORE_FLAG_IMAGE_FIXED: a 64-bit sum per pixel of every batch image
    in place of the splat buckets (the same size as the direct path plus
    8 bytes per pixel); it needs the PIXEL integrand and untiled runs."""
    direct = _pss_problem(R, n_chains=8192, flags=R.FLAG_SPLAT_DIRECT)
    fixed = _pss_problem(R, n_chains=8192, flags=R.FLAG_IMAGE_FIXED)
    nd = R.restore_state_bytes(direct.target, direct.mu, direct.local, direct.cfg)
    nf = R.restore_state_bytes(fixed.target, fixed.mu, fixed.local, fixed.cfg)
    n_pix = 64 * 64 * max(1, fixed.cfg.image_batches)
    assert 8 * n_pix <= nf - nd <= 8 * n_pix + 256
    p = _problem(R, flags=R.FLAG_IMAGE_FIXED)
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
    assert e.value.status == R.E_INVALID_ARG
    t = _pss_problem(R, n_chains=8192, flags=R.FLAG_IMAGE_FIXED, tile_px=16)
    with pytest.raises(R.RestoreError) as e:
        R.restore_state_bytes(t.target, t.mu, t.local, t.cfg)
    assert e.value.status == R.E_UNSUPPORTED


_TRACE_PROBE = """
import sys
sys.path.insert(0, {root!r})
from paper_2409_07148_amd import restore as R
from workloads import gmm_full
p = R.problem_from_workload(gmm_full(n_chains=1000))
n = R.restore_state_bytes(p.target, p.mu, p.local, p.cfg)
try:
    R.restore_init(p.target, p.mu, p.local, p.cfg, 256 + 4, n, stream=0)
except R.RestoreError as e:
    assert e.status == R.E_INVALID_ARG
print("roctx mapped:", "librocprofiler-sdk-roctx" in open("/proc/self/maps").read())
"""


@pytest.mark.parametrize("env,mapped", [("1", True), ("0", False), (None, False)])
def test_trace_ranges_open_roctx_only_when_asked(env, mapped):
    """RESTORE_TRACE=1 makes the first traced entry point (here restore_init
    with a misaligned state buffer, rejected before any device call) open
    the profiler SDK's roctx library; unset or 0 leaves it unloaded."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if not os.path.exists("/opt/rocm/lib/librocprofiler-sdk-roctx.so.1") and mapped:
        pytest.skip("no roctx library in this image")
    e = {k: v for k, v in os.environ.items() if k != "RESTORE_TRACE"}
    if env is not None:
        e["RESTORE_TRACE"] = env
    out = subprocess.run([sys.executable, "-c", _TRACE_PROBE.format(root=root)], capture_output=True, text=True,
                         env=e, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    assert f"roctx mapped: {mapped}" in out.stdout, out.stdout
