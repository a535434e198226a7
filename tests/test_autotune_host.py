"""Host logic of the schedule autotuner: cache round trip, selection, workload keys."""
import json

import numpy as np
import pytest

from paper_2405_02256_amd import autotune as AT


class _FakePlan:
    """Only what signature() reads: dims, counts, ndim, construction, num_images."""

    def __init__(self, dims, counts):
        self.dims = np.asarray(dims, np.int32)
        self.ndim = self.dims.shape[1]
        self.construction = 0
        self.num_images = len(self.dims)
        self._c = np.asarray(counts, np.int64)

    def counts(self):
        return self._c, self._c[:, : self._c.shape[1] // 2]


def test_pick_fastest_and_ties_keep_first():
    assert AT.pick({1: 3.0, 2: 1.0, 4: 2.0}) == 2
    assert AT.pick({512: 1.0, 1024: 1.0}) == 512
    assert AT.pick({}) is None


def test_cache_round_trip(tmp_path):
    c = AT.Cache(str(tmp_path / "sub" / "t.json"))
    assert c.get("dev", "sig") is None
    t = AT.Tuning(0, 4096, 2, 3, {"ect": {"1/0": 0.1}})
    c.put("dev", "sig", t)
    c.put("dev", "sig2", AT.Tuning(64, 2048, 0))
    c.put("dev2", "sig", AT.Tuning(0, 512, 8, 1))
    got = c.get("dev", "sig")
    assert got.as_args() == (0, 4096, 2, 3) and got.timings == {"ect": {"1/0": 0.1}}
    assert c.get("dev", "sig2").as_args() == (64, 2048, 0, 0)
    assert c.get("dev2", "sig").as_args() == (0, 512, 8, 1)
    assert set(json.load(open(c.path))) == {"dev", "dev2"}


def test_cache_tolerates_garbage(tmp_path):
    p = tmp_path / "t.json"
    p.write_text("{not json")
    c = AT.Cache(str(p))
    assert c.get("dev", "sig") is None
    c.put("dev", "sig", AT.Tuning())
    assert c.get("dev", "sig").as_args() == (0, 2048, 0, 0)
    p.write_text(json.dumps({"dev": {"sig": {"hybrid_chunk": "x"}}}))
    assert c.get("dev", "sig") is None


def test_signature_separates_workloads():
    a = _FakePlan([[512, 512]], [[10, 20, 30, 40]])
    b = _FakePlan([[512, 512]], [[10, 20, 30, 41]])
    base = AT.signature(a, 4096, 128, 4096, ("fourier",), "fp32", None)
    assert base == AT.signature(a, 4096, 128, 4096, ("fourier",), "fp32", None)
    assert base != AT.signature(b, 4096, 128, 4096, ("fourier",), "fp32", None)
    assert base != AT.signature(a, 4096, 64, 4096, ("fourier",), "fp32", None)
    assert base != AT.signature(a, 4096, 128, 4096, ("fourier", "laplace"), "fp32", None)
    assert base != AT.signature(a, 4096, 128, 4096, ("fourier",), "fp64", None)
    assert base != AT.signature(a, 4096, 128, 4096, ("fourier",), "fp32", "fourier")
    many = _FakePlan([[i + 2, 3] for i in range(20)], np.ones((20, 4)))
    assert "+12" in AT.signature(many)
