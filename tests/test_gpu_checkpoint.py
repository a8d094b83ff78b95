"""Checkpoint and resume of a resident state (bsim_state_save / load).

A state saved after some update batches and loaded into a new state must
give back the same summary, and the same update batches applied to the
original and to the loaded state must give equal results, each equal to the
oracle's batch summary of the updated graph (Theorem 2).  The file format
(header, sections, checksum) is rebuilt here independently, so a damaged
file with a valid checksum reaches the checks behind it."""

import struct

import numpy as np
import pytest

from oracle import oracle as orc
from oracle.updates import apply_ops
from paper_2111_12493_amd import binding
from paper_2111_12493_amd import graphgen as gg

from gpu_util import assert_same, ctx

pytestmark = pytest.mark.gpu

HEADER = struct.Struct("<8s6I4Q")
MASK = (1 << 64) - 1


def fold(chunks):
    acc = 0x243F6A8885A308D3
    for b in chunks:
        w = np.frombuffer(bytes(b) + b"\0" * ((-len(b)) % 8), dtype="<u8")
        for x in w.tolist():
            acc = ((acc ^ x) * 0x100000001B3) & MASK
    return acc


def split(data):
    """Header fields and the sections of a state file, in file order."""
    magic, version, k, flags, lb, n, _, m, nt, checksum, _ = HEADER.unpack_from(data, 0)
    sizes = [4 * (n + 1), 4 * m, lb * m, 4 * (n + 1), 4 * nt, n] + [8 * n] * (k + 1)
    pos, secs = HEADER.size, []
    for s in sizes:
        secs.append(bytearray(data[pos:pos + s]))
        pos += s
    assert pos == len(data)
    return dict(magic=magic, version=version, k=k, flags=flags, lb=lb, n=n, m=m, nt=nt,
                checksum=checksum), secs


def join(h, secs):
    head = HEADER.pack(h["magic"], h["version"], h["k"], h["flags"], h["lb"], h["n"], 0, h["m"], h["nt"],
                       fold(secs), 0)
    return head + b"".join(bytes(s) for s in secs)


def result_dict(r):
    d = r.to_dict()
    r.free()
    return d


def batches(g, rng, sizes, **kw):
    out = []
    for size in sizes:
        ops = gg.ops_as_tuples(gg.update_ops(g, rng, size, **kw))
        g = apply_ops(g, ops)
        out.append(ops)
    return out


@pytest.mark.parametrize("label_u16,stop,untyped", [(False, True, False), (True, False, False),
                                                     (False, False, True)])
def test_resume_gives_the_same_results(tmp_path, label_u16, stop, untyped):
    rng = np.random.default_rng(41)
    g = gg.uniform_graph(2000, 10000, 8, 16, seed=9)
    if label_u16:
        g = gg.with_u16_labels(g)
    k = 6 if stop else 4
    ops = batches(g, rng, [30, 300, 10, 1000, 3], n_labels=16, n_types=8)
    a = binding.State(ctx(), binding.HostGraph(g), k, stop_at_fixpoint=stop, untyped=untyped)
    last = result_dict(a.apply(binding.UpdateBatch(ops[0])))
    last = result_dict(a.apply(binding.UpdateBatch(ops[1])))
    g = apply_ops(apply_ops(g, ops[0]), ops[1])
    path = tmp_path / "state.bsim"
    a.save(path)
    assert not (tmp_path / "state.bsim.tmp").exists()
    b = binding.State.load(ctx(), path)
    assert_same(result_dict(b.result), last, "loaded summary")
    ga, gb = a.graph(), b.graph()
    for f in ("row_off", "tgt", "lab", "typ_off", "typ", "alive"):
        assert np.array_equal(getattr(ga, f), getattr(gb, f)), f
    for i, batch in enumerate(ops[2:]):
        g = apply_ops(g, batch)
        ra = result_dict(a.apply(binding.UpdateBatch(batch)))
        rb = result_dict(b.apply(binding.UpdateBatch(batch)))
        ref = orc.summarize(g, k, stop, untyped)
        assert_same(ra, ref, ("original", i))
        assert_same(rb, ref, ("loaded", i))
    a.free()
    b.free()


def test_small_and_edgeless_states(tmp_path):
    rng = np.random.default_rng(5)
    for trial, (n, m) in enumerate([(1, 0), (7, 0), (30, 90), (50, 400)]):
        g = gg.random_small_graph(rng, n, m, 3, 3, 3, p_alive=1.0 if trial % 2 else 0.8)
        for k in (0, 3):
            a = binding.State(ctx(), binding.HostGraph(g), k)
            path = tmp_path / ("s%d_%d" % (trial, k))
            a.save(path)
            b = binding.State.load(ctx(), path)
            assert_same(result_dict(b.result), orc.summarize(g, k, False, False), (n, m, k))
            a.free()
            b.free()


def make_file(tmp_path):
    rng = np.random.default_rng(8)
    g = gg.uniform_graph(300, 1500, 4, 6, seed=2)
    st = binding.State(ctx(), binding.HostGraph(g), 3)
    # delete two vertices so that the file holds dead ones
    st.apply(binding.UpdateBatch([("del_v", 5), ("del_v", 17)])).free()
    path = tmp_path / "good.bsim"
    st.save(path)
    st.free()
    return path.read_bytes()


def load_status(path):
    with pytest.raises(binding.BsimError) as e:
        binding.State.load(ctx(), path)
    return e.value.status


def test_format_and_damaged_files(tmp_path):
    data = make_file(tmp_path)
    h, secs = split(data)
    # the checksum rebuilt from the documented format agrees with the file
    assert h["magic"] == b"BSIMSTAT" and h["version"] == 1 and h["k"] == 3
    assert h["checksum"] == fold(secs)
    assert join(h, secs) == data
    alive = np.frombuffer(bytes(secs[5]), dtype=np.uint8)
    assert alive[5] == 0 and alive[17] == 0
    p = tmp_path / "bad.bsim"

    def status_of(blob):
        p.write_bytes(blob)
        return load_status(p)

    assert status_of(data[:-1]) == binding.E_INVALID                      # truncated
    assert status_of(data + b"\0") == binding.E_INVALID                   # trailing bytes
    assert status_of(b"XSIMSTAT" + data[8:]) == binding.E_INVALID         # magic
    assert status_of(data[:40]) == binding.E_INVALID                      # short header
    flipped = bytearray(data)
    flipped[-3] ^= 0x10                                                   # a level word
    assert status_of(bytes(flipped)) == binding.E_INVALID                 # checksum
    assert status_of(join({**h, "version": 2}, secs)) == binding.E_UNSUPPORTED
    # a valid checksum over a hash on a deleted vertex
    lv = [bytearray(s) for s in secs]
    word = np.frombuffer(bytes(lv[7]), dtype=np.uint64).copy()
    word[17] = 12345
    lv[7] = bytearray(word.tobytes())
    assert status_of(join(h, lv)) == binding.E_INVALID
    # a valid checksum over an edge target out of range: the graph checks
    tg = [bytearray(s) for s in secs]
    t = np.frombuffer(bytes(tg[1]), dtype=np.uint32).copy()
    t[0] = h["n"] + 3
    tg[1] = bytearray(t.tobytes())
    assert status_of(join(h, tg)) == binding.E_RANGE
    # offsets that disagree with the section sizes
    ro = [bytearray(s) for s in secs]
    r = np.frombuffer(bytes(ro[0]), dtype=np.uint32).copy()
    r[-1] -= 1
    ro[0] = bytearray(r.tobytes())
    assert status_of(join(h, ro)) == binding.E_INVALID
    assert load_status(tmp_path / "missing.bsim") == binding.E_IO
    # the intact file still loads after the failures
    p.write_bytes(data)
    binding.State.load(ctx(), p).free()


def test_save_to_an_unwritable_path(tmp_path):
    g = gg.uniform_graph(100, 300, 2, 3, seed=1)
    st = binding.State(ctx(), binding.HostGraph(g), 2)
    with pytest.raises(binding.BsimError) as e:
        st.save(tmp_path / "no_such_dir" / "s.bsim")
    assert e.value.status == binding.E_IO
    st.free()
