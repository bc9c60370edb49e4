"""The allocation-free entry point (fsm_mine_noalloc) against fsm_mine_ex.

It must return the same patterns and supports bit for bit, on two calls in a
row (the second with a smaller graph, over the scratch the first one left),
route nothing through the allocation hooks, and reject inputs beyond its
fixed scratch with a clear error -- after which it still works."""
import ctypes
import sys

import numpy as np
import pytest

import paper_2101_07690_amd as fsm
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class CountingHooks:
    """Allocation hooks that count calls and hand out torch memory."""

    def __init__(self):
        import torch
        self.calls = 0

        def _alloc(nbytes, _ctx):
            self.calls += 1
            return torch.cuda.caching_allocator_alloc(int(nbytes))

        def _release(ptr, _ctx):
            torch.cuda.caching_allocator_delete(ptr)

        self.hooks = (fsm._ALLOC_FN(_alloc), fsm._RELEASE_FN(_release))

    def __enter__(self):
        rc = fsm.lib().fsm_set_allocator(self.hooks[0], self.hooks[1], None)
        assert rc == 0
        return self

    def __exit__(self, *exc):
        fsm.lib().fsm_set_allocator(fsm._ALLOC_FN(), fsm._RELEASE_FN(), None)


def test_noalloc_matches_mine_ex_twice_smaller_second():
    w = synth.workload("er3300")
    big = (w["n"], w["src"], w["dst"], w["vertex_labels"])
    small = synth.tiny_graph(8300, 9, 14, 2)
    small = (len(small[2]), small[0], small[1], small[2])
    with fsm.Graph(*big) as gb, fsm.Graph(*small) as gs:
        want_big = fsm.mine(gb, 10, 5).patterns
        want_small = fsm.mine(gs, 1, 5).patterns
        with CountingHooks() as hooks:
            say("noalloc: er3300 t=10 sizes 2..5")
            got_big, st = fsm.mine_noalloc(gb, 10, 5)
            say("noalloc: tiny graph t=1 sizes 2..5")
            got_small, _ = fsm.mine_noalloc(gs, 1, 5)
            assert hooks.calls == 0
        assert got_big == want_big
        assert got_small == want_small
        assert st["levels"][5]["emitted"] > 0 and st["levels"][5]["kernel_ms"] == 0.0
        # the modes share the scratch the same way
        say("noalloc: vertex-induced, ST 2 sampling")
        assert fsm.mine_noalloc(gb, 10, 5, fsm.FSM_INDUCED)[0] == \
            fsm.mine(gb, 10, 5, fsm.FSM_INDUCED).patterns
        assert fsm.mine_noalloc(gb, 10, 5, join_threshold=2, seed=3)[0] == \
            fsm.mine(gb, 10, 5, join_threshold=2, seed=3).patterns


def test_noalloc_limits():
    w = synth.workload("er3300")
    args = (w["n"], w["src"], w["dst"], w["vertex_labels"])
    with fsm.Graph(*args) as g:
        want = fsm.mine(g, 10, 4).patterns
        # too small an output: the count is reported, nothing written
        o = fsm.Options()
        o.support, o.max_size, o.sampling_rate = 10, 4, 1.0
        cnt = ctypes.c_int64()
        rc = fsm.lib().fsm_mine_noalloc(g.handle, ctypes.byref(o), 3, None, None, None,
                                        ctypes.byref(cnt), None)
        assert rc == -1   # NULL arrays with capacity > 0
        sizes = np.zeros(3, np.int32)
        codes = np.zeros((3, 2 + fsm.MAX_SIZE), np.int32)
        sups = np.zeros(3, np.int64)
        rc = fsm.lib().fsm_mine_noalloc(
            g.handle, ctypes.byref(o), 3, sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            codes.ctypes.data_as(ctypes.POINTER(fsm.Code)),
            sups.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(cnt), None)
        assert rc == -4 and cnt.value == len(want)
        assert (sizes == 0).all()
    # a graph whose own state exceeds the scratch is rejected up front
    n = 5_000_000
    with fsm.Graph(n, [0], [1], np.zeros(n, np.int32)) as huge:
        with pytest.raises(fsm.FsmError) as e:
            fsm.mine_noalloc(huge, 1, 3)
        assert e.value.code == -4 and "scratch" in str(e.value)
    # a call that needs more than the scratch fails cleanly (or, if it fits,
    # agrees with fsm_mine_ex) ...
    cl = synth.workload("cl100k")
    with fsm.Graph(cl["n"], cl["src"], cl["dst"], cl["vertex_labels"]) as g:
        say("noalloc: cl100k (at or beyond the scratch)")
        try:
            got, _ = fsm.mine_noalloc(g, cl["support"], 5)
        except fsm.FsmError as e:
            assert e.code == -2 and "scratch" in str(e)
        else:
            assert got == fsm.mine(g, cl["support"], 5).patterns
    # ... and the next call still works
    with fsm.Graph(*args) as g:
        assert fsm.mine_noalloc(g, 10, 4)[0] == want
