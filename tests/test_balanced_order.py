"""The balanced domain order (LETKF_ORDER_BALANCED), host code of the
library, through a small C++ harness linked against it (no GPU).

Workgroup b of an analysis launch with one workgroup per domain runs on XCD
b % 8 and shares its CU with b +- num_cu (breadth-first dispatch).  The order
must be a permutation, keep every XCD's set of domains (the L2 locality of
the per-XCD order), put the costliest domains on CUs they have alone, and
not raise the estimated finish of the slowest CU.  With more domains than
resident workgroups (claimed as workgroups finish) it is longest first."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1310_5954_amd", "lib")
CSRC = os.path.join(ROOT, "paper_1310_5954_amd", "csrc")
SHARE = 0.15


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if not os.path.exists(os.path.join(LIBDIR, "libletkf.so")):
        pytest.skip("library not built")
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("bal") / "balanced_order")
    cmd = ["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}",
           "-I/opt/rocm/include", os.path.join(ROOT, "tests", "native", "balanced_order_main.cpp"),
           f"-L{LIBDIR}", "-lletkf", f"-Wl,-rpath,{LIBDIR}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def run(exe, cost, num_cu, resident=None):
    resident = 3 * num_cu if resident is None else resident
    inp = f"{len(cost)} {num_cu} {resident}\n" + " ".join(repr(float(c)) for c in cost) + "\n"
    r = subprocess.run([exe], input=inp, capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    xcd, bal = (np.array(line.split(), dtype=int) for line in r.stdout.strip().split("\n"))
    return xcd, bal


def makespan(order, cost, num_cu):
    """max over CUs of max + SHARE x (sum - max) of the costs placed on it"""
    cus = {}
    for b, l in enumerate(order):
        cus.setdefault(b % num_cu, []).append(cost[l])
    return max(max(v) + SHARE * (sum(v) - max(v)) for v in cus.values())


@pytest.mark.parametrize("n,num_cu", [(375, 256), (750, 256), (100, 256), (768, 256), (375, 80)])
def test_balanced_order_places_costly_domains_alone(harness, n, num_cu):
    rng = np.random.default_rng(n + num_cu)
    cost = 3.5 + rng.choice([7, 8, 8, 8, 9, 10, 11], size=n).astype(float)
    xcd, bal = run(harness, cost, num_cu, resident=max(n, 3 * num_cu))
    assert sorted(bal.tolist()) == list(range(n))
    # same domains on every XCD as the per-XCD order
    for x in range(8):
        assert sorted(bal[x::8].tolist()) == sorted(xcd[x::8].tolist())
    # sharing: how many positions fall on each position's CU
    per_cu = np.bincount(np.arange(n) % num_cu, minlength=num_cu)
    load = per_cu[np.arange(n) % num_cu]
    if load.min() < load.max():
        # on every XCD the costliest domains sit on its least shared CUs
        for x in range(8):
            b = np.arange(x, n, 8)
            lo = b[load[b] == load[b].min()]
            hi = b[load[b] > load[b].min()]
            if len(lo) and len(hi):
                assert cost[bal[lo]].max() >= cost[bal[hi]].max()
                assert np.sort(cost[bal[lo]])[::-1][0] == np.sort(cost[bal[b]])[::-1][0]
    assert makespan(bal, cost, num_cu) <= makespan(xcd, cost, num_cu) + 1e-9


def test_balanced_order_with_equal_costs_keeps_every_domain(harness):
    xcd, bal = run(harness, np.full(375, 5.0), 256)
    assert sorted(bal.tolist()) == list(range(375))
    for x in range(8):
        assert sorted(bal[x::8].tolist()) == sorted(xcd[x::8].tolist())


def test_balanced_order_falls_back_when_cus_do_not_split_over_xcds(harness):
    cost = np.arange(50, dtype=float)
    xcd, bal = run(harness, cost, 6, resident=64)  # 6 CUs: not a multiple of the 8 XCDs
    assert bal.tolist() == xcd.tolist()


def test_balanced_order_is_longest_first_beyond_the_resident_workgroups(harness):
    rng = np.random.default_rng(7)
    cost = 3.5 + rng.integers(8, 14, size=852).astype(float)
    _, bal = run(harness, cost, 256, resident=256)  # m = 128: one workgroup per CU
    assert sorted(bal.tolist()) == list(range(852))
    assert np.all(np.diff(cost[bal]) <= 0)
    # ties keep the map's order
    for c in np.unique(cost):
        idx = bal[cost[bal] == c]
        assert np.all(np.diff(idx) > 0)
