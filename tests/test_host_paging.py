"""Page replacement of streamed scenes (paper: the streaming module its
conclusion leaves to future work), host logic on the CPU.

The policy (paper_2505_06523_amd/csrc/page_lru.h) is driven through a small
C++ harness and checked on hand-worked sequences and against a plain
least-recently-used model written here: a cut keeps its resident clusters,
takes the least recently used pages for the missing ones, never evicts a
page of the same cut, refuses a cut larger than the pool without assigning
anything, and records the last-use frame of every evicted page.
"""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2505_06523_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("paging") / "paging_harness")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, os.path.join(HERE, "paging_harness.cpp"), "-o",
                    exe], check=True)
    return exe


class Run:
    def __init__(self, exe):
        self.p = subprocess.Popen([exe], stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)

    def cmd(self, line):
        self.p.stdin.write(line + "\n")
        self.p.stdin.flush()
        return self.p.stdout.readline().strip()

    def init(self, nc, npg):
        assert self.cmd("init %d %d" % (nc, npg)) == "init"

    def plan(self, ks):
        head, miss, pages, owners = self.cmd("plan " + " ".join(map(str, ks))).split("|")
        ok, touched, frame, maxst, ev = map(int, head.split())
        return dict(ok=bool(ok), touched=touched, frame=frame, max_evicted=maxst, evictions=ev,
                    miss=[int(x) for x in miss.split()], pages=[int(x) for x in pages.split()],
                    owners=[int(x) for x in owners.split()])

    def close(self):
        self.p.stdin.close()
        self.p.wait()


def test_hand_worked_sequence(harness):
    """Pool of 3 pages, clusters 0..9.  Initially page 0 is the least
    recently used (pages were listed 0, 1, 2 front-first in that order)."""
    r = Run(harness)
    r.init(10, 3)
    a = r.plan([4, 5])  # two misses take pages 0 and 1
    assert a["ok"] and a["miss"] == [4, 5] and a["pages"] == [0, 1] and a["evictions"] == 0
    b = r.plan([5, 6])  # 5 stays; 6 takes the free page 2
    assert b["touched"] == 1 and b["miss"] == [6] and b["pages"] == [2] and b["evictions"] == 0
    c = r.plan([7])  # the least recently used page is 4's (frame 1): evicted
    assert c["miss"] == [7] and c["pages"] == [0] and c["evictions"] == 1 and c["max_evicted"] == 1
    d = r.plan([6, 5, 8])  # 6 and 5 stay (touched); 8 takes 7's page (frame 3), not one of this cut
    assert d["touched"] == 2 and d["miss"] == [8] and d["pages"] == [0] and d["max_evicted"] == 3
    e = r.plan([1, 2, 3, 4])  # four clusters, three pages: refused, nothing assigned
    assert not e["ok"] and e["miss"] == [] and e["owners"] == d["owners"] and e["evictions"] == 2
    f = r.plan([5, 5, 5])  # repeats count once
    assert f["ok"] and f["touched"] == 1 and f["miss"] == []
    r.close()


def test_release_frees_a_page(harness):
    r = Run(harness)
    r.init(4, 2)
    a = r.plan([0, 1])
    assert r.cmd("release 1") == "release"
    b = r.plan([2])  # the freed page is taken without an eviction, whatever its place in the list
    assert b["miss"] == [2] and b["evictions"] == 0 and sorted(b["owners"]) == [0, 2]
    assert b["pages"] == [a["pages"][1]]  # the page 1 gave up
    r.close()


class RefLRU:
    """Plain model: a list of pages, most recently used first (a released
    page goes to the back)."""

    def __init__(self, nc, npg):
        self.order = list(range(npg))[::-1]  # pages listed front-first 0, 1, ... end with 0 at the back
        self.owner = [-1] * npg
        self.page = [-1] * nc
        self.stamp = [0] * npg
        self.frame = self.max_evicted = self.evictions = 0

    def plan(self, ks):
        self.frame += 1
        f = self.frame
        touched, miss = 0, []
        for k in ks:
            p = self.page[k]
            if p >= 0:
                if self.stamp[p] != f:
                    self.stamp[p] = f
                    self.order.remove(p)
                    self.order.insert(0, p)
                    touched += 1
            elif k not in miss:
                miss.append(k)
        if touched + len(miss) > len(self.owner):
            return False, touched, []
        for k in miss:
            p = self.order[-1]
            if self.owner[p] >= 0:
                self.page[self.owner[p]] = -1
                self.max_evicted = max(self.max_evicted, self.stamp[p])
                self.evictions += 1
            self.owner[p], self.page[k], self.stamp[p] = k, p, f
            self.order.remove(p)
            self.order.insert(0, p)
        return True, touched, miss

    def release(self, k):
        p = self.page[k]
        if p >= 0:
            self.owner[p], self.page[k] = -1, -1
            self.order.remove(p)
            self.order.append(p)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_cuts_match_the_model(harness, seed):
    """300 random cuts (sizes 1..40, some larger than the pool) over 200
    clusters and a 32-page pool: every decision equals the model's, and a
    cut's clusters are all resident after it is accepted."""
    rng = np.random.default_rng(seed)
    r = Run(harness)
    r.init(200, 32)
    ref = RefLRU(200, 32)
    hot = rng.choice(200, 60, replace=False)
    for i in range(300):
        n = int(rng.integers(1, 41))
        ks = [int(x) for x in (rng.choice(hot, n) if rng.random() < 0.7 else rng.integers(0, 200, n))]
        got = r.plan(ks)
        ok, touched, miss = ref.plan(ks)
        assert got["ok"] == ok and got["touched"] == touched and got["miss"] == miss, (i, got, ok, touched, miss)
        assert got["owners"] == ref.owner and got["evictions"] == ref.evictions
        assert got["max_evicted"] == ref.max_evicted and got["frame"] == ref.frame
        if ok:
            assert set(ks) <= set(o for o in got["owners"] if o >= 0)
        if rng.random() < 0.05:  # now and then a page whose contents failed to arrive
            k = int(rng.integers(0, 200))
            r.cmd("release %d" % k)
            ref.release(k)
    r.close()


# --------------------------------------------------------------------------
# page images of a streamed scene: host memory or a file on disk
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def store_harness(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("store") / "page_store_harness")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", CSRC, os.path.join(HERE, "page_store_harness.cpp"),
                    "-o", exe], check=True)
    return exe


def _store(exe, path, n, page_bytes, direct):
    p = subprocess.Popen([exe, path, str(n), str(page_bytes), str(int(direct))], stdin=subprocess.PIPE,
                         stdout=subprocess.PIPE, text=True)
    head = p.stdout.readline().split()
    assert head[0] == "ready", head
    return p, int(head[1]), int(head[2])


def _get(p, ks):
    p.stdin.write("get " + " ".join(map(str, ks)) + "\n")
    p.stdin.flush()
    head, same, pad = p.stdout.readline().split("|")
    ok, tier, reads = map(int, head.split())
    return ok, tier, reads, [int(x) for x in same.split()], int(pad)


@pytest.mark.parametrize("where,direct", [("memory", False), ("file", False), ("file", True)])
def test_page_store_round_trip(store_harness, tmp_path, where, direct):
    """Every image comes back exactly, in the order asked, at the store's
    stride (4 KiB-aligned slots for a file), with one read per run of
    consecutive clusters from a file; nothing past the batch is written."""
    path = "-" if where == "memory" else str(tmp_path / "pages.bin")
    page_bytes = 15104  # a 64-row SH3 FP32 page image
    p, tier, stride = _store(store_harness, path, 40, page_bytes, direct)
    if where == "memory":
        assert tier == 0 and stride == page_bytes
    else:
        assert tier in ((2, 1) if direct else (1,)) and stride == 16384
        assert os.path.getsize(path) == 40 * 16384
    ok, _, r0, same, pad = _get(p, [0, 1, 2, 7, 8, 20, 39])
    assert ok and same == [1] * 7 and pad == 1
    if where == "file":
        assert r0 == 4  # runs 0-2, 7-8, 20, 39
    ok, _, r1, same, pad = _get(p, list(range(10, 30)))
    assert ok and same == [1] * 20 and pad == 1
    if where == "file":
        assert r1 - r0 == 1
    p.stdin.close()
    p.wait()
    if where == "file":
        assert not os.path.exists(path)  # removed with the store


def test_blend_plan_bounds(tmp_path):
    """The chunk-record bound the runtime sizes its buffers by
    (paper_2505_06523_amd/csrc/blend_plan.h) holds on random plans: at that
    size every long bin list is chunked for each of its tiles, and at any size
    the records handed out, the work items and the re-walk entries stay inside
    the buffer; the chunks of a list tile it exactly (C++ harness, CPU)."""
    exe = str(tmp_path / "plan_harness")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-I", CSRC, os.path.join(HERE, "plan_harness.cpp"), "-o",
                    exe], check=True)
    out = subprocess.run([exe, "1500"], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok 1500", out.stdout + out.stderr


def test_chunk_sizes_read_from_the_plan_header():
    """The GPU tests size their long lists from the plan header's chunk sizes."""
    from tests import helpers as H
    for server in (False, True):
        first, later = H.blend_chunk_sizes(server)
        assert 1024 <= later <= 4096 and first == 3 * later
    assert H.blend_chunk_sizes(True)[1] >= H.blend_chunk_sizes(False)[1]
