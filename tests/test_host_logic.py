"""Host-side logic of the library that needs no GPU, compiled and run here."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run_cpp(src):
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "check")
        subprocess.run(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17",
                        "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_1701_04733_amd", "csrc"),
                        os.path.join(ROOT, "tests", "cpp", src), "-o", exe],
                       check=True, capture_output=True, timeout=300)
        return subprocess.run([exe], capture_output=True, text=True, timeout=120)


def test_tile_plans_cover_every_output_once():
    r = _run_cpp("tile_plan_check.cpp")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "tile plan failures: 0" in r.stdout


def test_floyd_warshall_schedule_keeps_the_blocked_order():
    """Pairs and groups of four pivot blocks, nb = 1..40 and 256: every block
    gets every pivot block's update once, in order, from operands in the
    blocked order's state, and no launch writes a block it reads."""
    r = _run_cpp("fw_schedule_check.cpp")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "fw schedule failures: 0" in r.stdout


def test_pool_allocator_never_overlaps_and_coalesces():
    r = _run_cpp("range_alloc_check.cpp")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "range allocator failures: 0" in r.stdout


# ---- the single launch's tagged ordering, simulated on the host ----------
# A model of the tagged mode of the single-launch APSP solve: one workgroup
# per tile of an nt x nt grid; squaring t of tile (I, J) needs D_{t-1} of
# every tile of row panel I and column panel J, read from matrix (t-1) mod B
# of a ring of B tagged matrices (the kernel uses B = 2), and writes its tile
# of D_t, tagged t, to matrix t mod B.  Workgroups advance one memory access at a time in an
# adversarial random order (all of them resident, as in a cooperative
# launch); a read whose tag is not the expected one is retried.  Early exit:
# each workgroup publishes a change word per squaring and, after squaring t,
# waits for every workgroup's word of squaring t - 1; none changed -> stop
# with step count t - 1.

def _simulate_tagged(nt, T, ring, fixpoint, seed, early):
    import random
    rnd = random.Random(seed)
    tiles = [(i, j) for i in range(nt) for j in range(nt)]
    mats = [dict() for _ in range(ring)]            # (tile) -> (tag, version)
    for q in tiles:
        mats[0][q] = (0, (q, 0))
    words = {}                                      # (step, tile) -> changed bit
    # changed(tile, t): some tile changes at every squaring before the fixpoint
    changed = {}
    for t in range(1, T + 1):
        if t < fixpoint:
            hit = rnd.choice(tiles)
            for q in tiles:
                changed[(q, t)] = (q == hit) or rnd.random() < 0.3
        else:
            for q in tiles:
                changed[(q, t)] = False
    result = {}

    def program(me):
        I, J = me
        need = sorted({(I, j) for j in range(nt)} | {(i, J) for i in range(nt)})
        steps = 0
        for t in range(1, T + 1):
            src = mats[(t - 1) % ring]
            for q in need:
                while True:
                    tag, ver = src.get(q, (-1, None))
                    if tag == t - 1:
                        assert ver == (q, t - 1), ("stale data", me, q, t, ver)
                        break
                    assert tag < t - 1 or tag == -1, ("overwritten before read", me, q, t, tag)
                    yield "spin"
                yield "read"
            steps = t
            if t < T:
                mats[t % ring][me] = (t, (me, t))
                yield "write"
            if early:
                words[(t, me)] = changed[(me, t)]
                yield "word"
                if t >= 2:
                    any_changed = False
                    for q in tiles:
                        while (t - 1, q) not in words:
                            yield "spin"
                        any_changed |= words[(t - 1, q)]
                        yield "read"
                    if not any_changed:
                        steps = t - 1
                        break
        result[me] = steps

    live = {q: program(q) for q in tiles}
    idle_rounds = 0
    while live:
        progressed = False
        for q in rnd.sample(list(live), len(live)):
            for _ in range(rnd.randint(1, 3)):
                try:
                    what = next(live[q])
                except StopIteration:
                    del live[q]
                    progressed = True
                    break
                if what != "spin":
                    progressed = True
        idle_rounds = 0 if progressed else idle_rounds + 1
        if idle_rounds > 50:
            return None                             # every live workgroup waits: deadlock
    return result


def test_tagged_single_launch_ordering_two_matrices():
    """A ring of two tagged matrices (the kernel's) and of three: under random
    schedules every read that passes the tag check gets the intended D_{t-1}
    tile, nothing is overwritten before its last reader, the launch never
    deadlocks, and with early exit every workgroup stops with the barrier
    path's step count."""
    for seed in range(40):
        nt = 2 + seed % 4
        T = 2 + seed % 6
        fixpoint = 1 + seed % (T + 2)               # 1..T+1: also "never within T"
        for ring in (2, 3):
            for early in (False, True):
                res = _simulate_tagged(nt, T, ring, fixpoint, seed, early)
                assert res is not None, ("deadlock", seed, ring, early)
                want = T if not early else (fixpoint if fixpoint <= T else T)
                assert set(res.values()) == {want}, (seed, ring, early, res, want)


def test_tagged_ordering_model_detects_a_short_ring():
    """The model is sensitive: with a single matrix some schedule overwrites
    a tile that a lagging workgroup has not read yet."""
    failures = 0
    for seed in range(100):
        try:
            if _simulate_tagged(3, 6, 1, 99, seed, False) is None:
                failures += 1
        except AssertionError:
            failures += 1
    assert failures > 0
