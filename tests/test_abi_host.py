"""Host-side checks of the C ABI: the library loads, exports every function
include/snlm.h declares, and rejects bad jobs before touching a device."""
import math
import os
import re

import pytest

import paper_1407_2343_amd as snlm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "snlm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(snlm_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("snlm_create", "snlm_destroy", "snlm_denoise", "snlm_denoise_ex",
                     "snlm_denoise_batch", "snlm_enqueue_ex", "snlm_enqueue_batch",
                     "snlm_submit", "snlm_submit_many", "snlm_poll", "snlm_job_device_ms",
                     "snlm_sync", "snlm_workspace_bytes", "snlm_serving_bytes",
                     "snlm_strerror", "snlm_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = snlm.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_and_version():
    assert snlm.strerror(0) == "ok"
    assert "arena" in snlm.strerror(-2)
    assert snlm.strerror(12345) == "unknown status"
    assert "gfx950" in snlm.version()


def test_workspace_bytes():
    assert snlm.workspace_bytes(512, 512) == 512 * 512 * 4
    assert snlm.workspace_bytes(3, 5) == 256  # rounded to 256 bytes
    assert snlm.workspace_bytes(0, 5) == 0


def test_serving_bytes_cover_input_intermediate_and_output():
    L = snlm.lib()
    # 100 x 70: FP32 input 28000 B -> 28160, intermediate 100 x 80 x 4 = 32000 -> 32000,
    # output 28000 -> 28160
    assert L.snlm_serving_bytes(100, 70, 0) == 28160 + 32000 + 28160
    # FP16 input: 14000 -> 14080
    assert L.snlm_serving_bytes(100, 70, 1) == 14080 + 32000 + 28160
    assert L.snlm_serving_bytes(0, 70, 0) == 0
    assert snlm.strerror(snlm.EBUSY) == "served jobs hold the arena"


GOOD = dict(img=0x100000, out=0x900000, H=64, W=80, S=10, K=3, h=200.0)


def job(**kw):
    d = dict(GOOD)
    d.update(kw)
    return snlm.make_job(**d)


def test_valid_job_passes():
    assert snlm.validate(job())[0] == snlm.OK
    assert snlm.validate(job(h=math.inf))[0] == snlm.OK
    assert snlm.validate(job(S=0, K=0))[0] == snlm.OK
    assert snlm.validate(job(S=16, K=8, kernel="gauss"))[0] == snlm.OK
    assert snlm.validate(job(dtype="f16", sum="kahan"))[0] == snlm.OK


@pytest.mark.parametrize("bad,reason", [
    (dict(img=0), "non-NULL"),
    (dict(out=0), "non-NULL"),
    (dict(H=0), ">= 1"),
    (dict(W=-3), ">= 1"),
    (dict(ld_in=10), "pitches"),
    (dict(ld_out=79), "pitches"),
    (dict(S=17), "S out of range"),
    (dict(S=-1), "S out of range"),
    (dict(K=9), "K out of range"),
    (dict(h=0.0), "h must be"),
    (dict(h=-1.0), "h must be"),
    (dict(h=float("nan")), "h must be"),
    (dict(seg_len=20), "multiple of 16"),
    (dict(out=0x100000 + 100), "overlaps"),
    (dict(H=40000, W=40000), "2 GiB"),
])
def test_invalid_jobs_rejected(bad, reason):
    rc, why = snlm.validate(job(**bad))
    assert rc == snlm.EINVAL
    assert reason in why


def test_recursive_gaussian_rules():
    ok = lambda **kw: snlm.validate(job(kernel="gauss_iir", **kw))
    assert ok(beta=0.5)[0] == snlm.OK
    assert ok(beta=256.0)[0] == snlm.OK
    assert ok(K=1)[0] == snlm.OK  # default beta = K / 2
    for kw in (dict(beta=0.49), dict(beta=256.5), dict(K=0)):
        rc, why = ok(**kw)
        assert rc == snlm.EINVAL and "0.5 <= beta" in why, kw
    # a pass stores 3 S ((n + L - 1) / 16 + 2) FP64 forward states per line,
    # L = ceil(6 beta) + S + 3: a 16000 x 16000 image at S = 16 needs 6 GiB
    big = dict(img=0x100000, out=0x100000 + 2 * 16000 * 16000 * 4, H=16000, W=16000, S=16, beta=8.0)
    rc, why = ok(**big)
    assert rc == snlm.EINVAL and "2 GiB" in why
    assert snlm.validate(job(**dict(big, kernel="gauss", K=8)))[0] == snlm.OK
    # at S = 16, beta = 2 the largest square image is 9430 x 9430 (2.147e9
    # bytes of states, just below 2^31 - 1)
    for n, want in ((9430, snlm.OK), (9440, snlm.EINVAL)):
        states = 3 * 16 * ((n + 31 - 1) // 16 + 2) * n * 8
        assert (states < 2 ** 31 - 1) == (want == snlm.OK)
        edge = dict(img=0x100000, out=0x100000 + 2 * n * n * 4, H=n, W=n, S=16, beta=2.0)
        assert ok(**edge)[0] == want, n


def test_unknown_enums_rejected():
    j = job()
    j.kernel = 7
    assert snlm.validate(j)[0] == snlm.EINVAL
    j = job()
    j.order = 2
    assert snlm.validate(j)[0] == snlm.EINVAL
    j = job()
    j.sum = 9
    assert snlm.validate(j)[0] == snlm.EINVAL
    j = job()
    j.dtype = 3
    assert snlm.validate(j)[0] == snlm.EINVAL


def test_null_context_calls_are_rejected():
    lib = snlm.lib()
    j = job()
    import ctypes
    assert lib.snlm_denoise_ex(None, ctypes.byref(j)) == snlm.EINVAL
    assert lib.snlm_sync(None) == snlm.EINVAL
    assert lib.snlm_poll(None, 1) == snlm.EINVAL
    assert lib.snlm_destroy(None) == snlm.OK
    assert lib.snlm_create(None, 0, None, None, 0) == snlm.EINVAL


def test_sure_and_volume_workspaces():
    H, W = 100, 37
    off = snlm.sure_layout(H, W)
    plane = snlm.workspace_bytes(H, W)
    assert off[:5] == [k * plane for k in range(5)]
    assert off[5] == 5 * plane and off[6] > off[5] and off[7] > off[6]
    assert snlm.sure_workspace_bytes(H, W) == off[7]
    assert snlm.full_workspace_bytes(H, W) == off[7] + plane
    assert snlm.sure_workspace_bytes(0, 5) == 0 and snlm.full_workspace_bytes(5, 0) == 0
    Wp = (W + 15) // 16 * 16
    assert snlm.workspace3d_bytes(3, H, W) >= 2 * 3 * H * Wp * 4
    assert snlm.workspace3d_bytes(0, H, W) == 0
    with pytest.raises(snlm.SnlmError):
        snlm.sure_layout(0, 3)


def test_bilateral_params_follow_the_rules():
    import oracle
    for s in (5.0, 15.0, 20.0, 30.0, 50.0):
        a, b = snlm.bilateral_params(s)
        ra, rb = oracle.bf_params(s)
        assert a == pytest.approx(ra, rel=1e-6) and b == pytest.approx(rb, rel=1e-6)
