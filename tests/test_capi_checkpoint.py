"""Training checkpoints of the learned column decision (rl0_mlp_save / rl0_mlp_load) on the
host: files written here from the layout the header documents (Python's struct and zlib,
not the library) are read back through rl0_mlp_load without device arrays, and every
check that guards a load (magic, version, checksums of header and payload, dtype, d and
P, size, hyper-parameters) rejects a spoiled file with RL0_EIO before anything is
written.  The round trip through device memory and the exact resume of training run on
the GPU (test_gpu_mlp.py)."""
import ctypes
import struct
import zlib

import numpy as np
import pytest

R = pytest.importorskip("paper_1704_09012_amd.rl0")

D, SEED, STEP = 7, 12345, 300
HP = (1e-3, 0.9, 0.999, 1e-8, 0.5)
BATCH = 2048


def payload(P, seed=0):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(P).astype("<f4")
    m = (rng.standard_normal(P) * 1e-3).astype("<f4")
    v = (rng.random(P) * 1e-6).astype("<f4")
    return w.tobytes() + m.tobytes() + v.tobytes()


def header(P, body, *, magic=b"RL0MLPCK", version=1, dtype=0, d=D, batch=BATCH, seed=SEED, step=STEP, hp=HP,
           body_crc=None, reserved=0, head_crc=None):
    h = magic + struct.pack("<IIiiqQq5f", version, dtype, d, batch, P, seed, step, *hp)
    h += struct.pack("<I", zlib.crc32(body) if body_crc is None else body_crc)
    assert len(h) == 72
    h += struct.pack("<II", zlib.crc32(h) if head_crc is None else head_crc, reserved)
    return h


def write(tmp_path, blob, name="ck.bin"):
    p = tmp_path / name
    p.write_bytes(blob)
    return str(p)


def test_layout_reads_back(tmp_path):
    P = R.mlp_num_params(D)
    body = payload(P)
    info = R.mlp_checkpoint_info(write(tmp_path, header(P, body) + body))
    assert info["d"] == D and info["P"] == P and info["dtype"] == 0
    assert info["seed"] == SEED and info["step"] == STEP
    cfg = info["cfg"]
    assert cfg["batch"] == BATCH and cfg["t0"] == STEP and cfg["steps"] == 0
    got = (cfg["lr"], cfg["beta1"], cfg["beta2"], cfg["eps"], cfg["lam"])
    assert got == tuple(float(np.float32(x)) for x in HP)


def test_header_is_80_bytes_and_payload_follows(tmp_path):
    P = R.mlp_num_params(3)
    body = payload(P, 1)
    blob = header(P, body, d=3) + body
    assert len(blob) == 80 + 12 * P
    assert R.mlp_checkpoint_info(write(tmp_path, blob))["P"] == P


@pytest.mark.parametrize("spoil", [
    "magic", "version", "header_crc", "reserved", "dtype", "d_zero", "d_big", "P", "step", "batch", "lr_nan",
    "truncated", "trailing", "payload_crc", "flipped_byte", "short_header", "empty",
])
def test_spoiled_files_are_rejected(tmp_path, spoil):
    P = R.mlp_num_params(D)
    body = payload(P)
    kw = {}
    if spoil == "magic":
        kw["magic"] = b"RL0MLPCX"
    elif spoil == "version":
        kw["version"] = 2
    elif spoil == "header_crc":
        kw["head_crc"] = 0
    elif spoil == "reserved":
        kw["reserved"] = 1
    elif spoil == "dtype":
        kw["dtype"] = 1
    elif spoil == "d_zero":
        kw["d"] = 0
    elif spoil == "d_big":
        kw["d"] = 17
    elif spoil == "P":
        P_bad = P + 1
    elif spoil == "step":
        kw["step"] = -1
    elif spoil == "batch":
        kw["batch"] = 0
    elif spoil == "lr_nan":
        kw["hp"] = (float("nan"),) + HP[1:]
    elif spoil == "payload_crc":
        kw["body_crc"] = zlib.crc32(body) ^ 1
    blob = header(P_bad if spoil == "P" else P, body, **kw) + body
    if spoil == "truncated":
        blob = blob[:-4]
    elif spoil == "trailing":
        blob = blob + b"\0"
    elif spoil == "flipped_byte":
        b = bytearray(blob)
        b[80 + 5 * P + 2] ^= 0x10
        blob = bytes(b)
    elif spoil == "short_header":
        blob = blob[:79]
    elif spoil == "empty":
        blob = b""
    with pytest.raises(R.Rl0Error) as e:
        R.mlp_checkpoint_info(write(tmp_path, blob))
    assert e.value.code == -7 and "checkpoint" in str(e.value)


def test_missing_file(tmp_path):
    with pytest.raises(R.Rl0Error) as e:
        R.mlp_checkpoint_info(str(tmp_path / "absent.bin"))
    assert e.value.code == -7


def test_a_rejected_load_writes_nothing(tmp_path):
    """The checks run on the whole file before any copy: a spoiled payload leaves the
    caller's info struct as it was (and would leave device arrays alone)."""
    P = R.mlp_num_params(D)
    body = payload(P)
    path = write(tmp_path, header(P, body, body_crc=0) + body)
    info = R.MlpCkpt(d=-99)
    rc = R.lib().rl0_mlp_load(path.encode(), ctypes.byref(info), None, None, None, None)
    assert rc == -7 and info.d == -99 and b"payload checksum" in R.lib().rl0_last_error()


def test_save_checks_its_arguments(tmp_path):
    """Bad arguments are refused before any device copy (so no GPU is needed here)."""
    L = R.lib()
    fake = ctypes.c_void_p(0x1000)
    path = str(tmp_path / "ck.bin").encode()
    good = R.MlpCkpt(D, 0, 0, 1, 5, R.TrainCfg(*HP, BATCH, 0, 0))
    for bad in (R.MlpCkpt(0, 0, 0, 1, 5, good.cfg), R.MlpCkpt(D, 0, 0, 1, -1, good.cfg),
                R.MlpCkpt(D, 0, 0, 1, 5, R.TrainCfg(float("inf"), 0.9, 0.999, 1e-8, 1.0, BATCH, 0, 0)),
                R.MlpCkpt(D, 0, 0, 1, 5, R.TrainCfg(*HP, 0, 0, 0))):
        assert L.rl0_mlp_save(path, ctypes.byref(bad), fake, fake, fake, None) == -1
    assert L.rl0_mlp_save(path, ctypes.byref(good), None, fake, fake, None) == -1
    assert L.rl0_mlp_save(None, ctypes.byref(good), fake, fake, fake, None) == -1
    assert not (tmp_path / "ck.bin").exists() and not (tmp_path / "ck.bin.tmp").exists()
