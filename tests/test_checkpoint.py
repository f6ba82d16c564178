"""Checkpoint and resume of load stepping, on the CPU with a stand-in load step (a
deterministic, history-dependent update of u), so that a resumed run must reproduce
the uninterrupted one bit for bit."""
import os

import numpy as np
import pytest
import torch

from paper_2204_01722_amd import checkpoint


def _step(k, u):
    u.mul_(0.9).add_(torch.sin(u + k)).add_(0.1 * k)
    return {"level": k, "norm": float(u.norm())}


def _u0():
    g = torch.Generator().manual_seed(3)
    return torch.randn(17, 3, generator=g, dtype=torch.float64)


def _full(n):
    u = _u0()
    for k in range(1, n + 1):
        _step(k, u)
    return u


def test_uninterrupted_run_writes_every_level(tmp_path):
    path = str(tmp_path / "ck.npz")
    u, first, level, stats = checkpoint.run_load_steps(_step, _u0(), 5, path, tag="a")
    assert (first, level) == (1, 5)
    assert [s["level"] for s in stats] == [1, 2, 3, 4, 5]
    assert torch.equal(u, _full(5))
    saved, lv = checkpoint.load(path, (17, 3), 5, "a")
    assert lv == 5 and np.array_equal(saved, u.numpy())
    assert os.listdir(tmp_path) == ["ck.npz"]  # no temporary left behind
    # a finished run given its own checkpoint has nothing left to do
    u2, first, level, stats = checkpoint.run_load_steps(_step, _u0(), 5, path, tag="a")
    assert (first, level, stats) == (6, 5, []) and torch.equal(u2, u)


def test_stop_and_resume_reproduce_the_full_run(tmp_path):
    path = str(tmp_path / "ck.npz")
    u, first, level, _ = checkpoint.run_load_steps(_step, _u0(), 6, path, tag="b", stop_after=2)
    assert (first, level) == (1, 2)
    u, first, level, _ = checkpoint.run_load_steps(_step, torch.zeros(17, 3, dtype=torch.float64), 6, path,
                                                   tag="b", stop_after=4)
    assert (first, level) == (3, 4)
    u, first, level, stats = checkpoint.run_load_steps(_step, torch.zeros(17, 3, dtype=torch.float64), 6,
                                                       path, tag="b")
    assert (first, level) == (5, 6) and [s["level"] for s in stats] == [5, 6]
    assert torch.equal(u, _full(6))


def test_resume_after_a_failed_level(tmp_path):
    path = str(tmp_path / "ck.npz")

    def failing(k, u):
        if k == 4:
            raise RuntimeError("level 4 did not converge")
        return _step(k, u)

    with pytest.raises(RuntimeError, match="level 4"):
        checkpoint.run_load_steps(failing, _u0(), 5, path, tag="c")
    assert checkpoint.load(path, (17, 3), 5, "c")[1] == 3
    u, first, level, _ = checkpoint.run_load_steps(_step, _u0(), 5, path, tag="c")
    assert (first, level) == (4, 5)
    assert torch.equal(u, _full(5))


def test_foreign_checkpoints_are_rejected(tmp_path):
    path = str(tmp_path / "ck.npz")
    checkpoint.run_load_steps(_step, _u0(), 4, path, tag="d", stop_after=1)
    with pytest.raises(ValueError, match="load steps"):
        checkpoint.run_load_steps(_step, _u0(), 5, path, tag="d")
    with pytest.raises(ValueError, match="another problem"):
        checkpoint.run_load_steps(_step, _u0(), 4, path, tag="e")
    with pytest.raises(ValueError, match="shape"):
        checkpoint.run_load_steps(_step, torch.zeros(16, 3, dtype=torch.float64), 4, path, tag="d")
    with pytest.raises(ValueError):
        checkpoint.run_load_steps(_step, _u0(), 0, None)


def test_fingerprint_tells_problems_apart():
    a = torch.arange(12, dtype=torch.float64).reshape(4, 3)
    b = a.clone()
    b[2, 1] += 1e-12
    assert checkpoint.fingerprint(a, None) == checkpoint.fingerprint(a.clone(), None)
    assert checkpoint.fingerprint(a, None) != checkpoint.fingerprint(b, None)
    assert checkpoint.fingerprint(a, None) != checkpoint.fingerprint(a, a)
    assert checkpoint.fingerprint(a, None, extra="x") != checkpoint.fingerprint(a, None, extra="y")


def test_a_failed_write_keeps_the_previous_checkpoint(tmp_path, monkeypatch):
    path = str(tmp_path / "ck.npz")
    checkpoint.run_load_steps(_step, _u0(), 4, path, tag="f", stop_after=2)
    real = np.savez

    def broken(file, **arrays):
        real(file, **arrays)
        raise OSError("disk full")

    monkeypatch.setattr(checkpoint.np, "savez", broken)
    with pytest.raises(OSError, match="disk full"):
        checkpoint.run_load_steps(_step, _u0(), 4, path, tag="f")
    monkeypatch.undo()
    assert os.listdir(tmp_path) == ["ck.npz"]
    assert checkpoint.load(path, (17, 3), 4, "f")[1] == 2
    u, first, level, _ = checkpoint.run_load_steps(_step, _u0(), 4, path, tag="f")
    assert (first, level) == (3, 4) and torch.equal(u, _full(4))
