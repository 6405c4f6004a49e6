"""Host-side models of the two protocols by which the workgroups of one pair
meet in the multi-workgroup launches, checked over random interleavings of
their steps (sequentially consistent: the kernels get the same order from
agent-scope release and acquire).

* The split layout (two workgroups per pair): before every exchange event
  k a half raises its counter to k (its data written first), then waits for
  the partner's counter to reach k.  A wait that gives up (the model lets
  any wait give up while the partner has not arrived, as a wait does after
  its time limit) writes the half's failure word, sets its flag, and every
  later wait of that half returns at once.  At the end both raise the final
  event; half 1 stops there, half 0 waits for it and then reads half 1's
  failure word.  Claims: every run ends; without a give-up every wait
  returns after the partner's raise of the same event; with any give-up,
  half 0 reports the pair lost.
* The group launch (G workgroups per pair, B barriers): at each barrier a
  workgroup adds one to the pair's counter and waits for G times the
  barriers so far, with the same give-up rule, writing the pair's failure
  word when it gives up.  Workgroup 0 reads that word after its last
  barrier.  Claims: every run ends; without a give-up no workgroup leaves a
  barrier before all have reached it; a give-up at any barrier but the last
  (after which a workgroup other than 0 only returns) is reported.  After a
  give-up the others may pass later barriers early (the workgroup that gave
  up raises the counter without waiting), so the data of that pair is not to
  be trusted, which its status says; the kernels keep every address
  independent of such data (pivot indices read from memory are masked into
  range)."""
import random

import pytest


def _run_split(n_events, rng, p_give_up):
    cnt = [0, 0]
    fail_word = [False, False]
    flag = [False, False]
    early = []  # waits that returned before the partner's raise (give-ups excluded)
    status = None

    def half(h):
        nonlocal status
        for k in range(1, n_events + 1):
            cnt[h] = k
            yield
            while not flag[h] and cnt[1 - h] < k:
                if rng.random() < p_give_up:
                    fail_word[h] = True
                    flag[h] = True
                    break
                yield
            if not flag[h] and cnt[1 - h] < k:
                early.append((h, k))
            yield
        cnt[h] = n_events + 1
        yield
        if h == 1:
            return
        while not flag[0] and cnt[1] < n_events + 1:
            if rng.random() < p_give_up:
                fail_word[0] = True
                flag[0] = True
                break
            yield
        status = "lost" if (flag[0] or fail_word[1]) else "ok"

    procs = [half(0), half(1)]
    steps = 0
    while procs:
        p = rng.choice(procs)
        try:
            next(p)
        except StopIteration:
            procs.remove(p)
        steps += 1
        assert steps < 100000, "the model did not end"
    return status, fail_word, early


@pytest.mark.parametrize("p_give_up", [0.0, 0.02, 0.2])
def test_split_exchange_reports_every_give_up(p_give_up):
    rng = random.Random(7)
    for _ in range(2000):
        status, fail_word, early = _run_split(rng.randint(1, 6), rng, p_give_up)
        assert not early
        if any(fail_word):
            assert status == "lost"
        elif p_give_up == 0.0:
            assert status == "ok"


def _run_group(G, B, rng, p_give_up):
    cnt = [0]
    fail_word = [False]
    flag = [False] * G
    arrived = [0] * G        # barriers each workgroup has reached
    violations = []
    gave_up_at = []
    report = None

    def wg(g):
        nonlocal report
        for b in range(1, B + 1):
            arrived[g] = b
            cnt[0] += 1
            yield
            while not flag[g] and cnt[0] < G * b:
                if rng.random() < p_give_up:
                    fail_word[0] = True
                    flag[g] = True
                    gave_up_at.append((g, b))
                    break
                yield
            if not flag[g] and min(arrived) < b:
                violations.append((g, b))
            yield
        if g == 0:
            report = "lost" if (flag[0] or fail_word[0]) else "ok"

    procs = [wg(g) for g in range(G)]
    steps = 0
    while procs:
        p = rng.choice(procs)
        try:
            next(p)
        except StopIteration:
            procs.remove(p)
        steps += 1
        assert steps < 200000, "the model did not end"
    return report, gave_up_at, violations


@pytest.mark.parametrize("p_give_up", [0.0, 0.02, 0.2])
def test_group_barrier_reports_give_ups_before_the_last(p_give_up):
    rng = random.Random(11)
    for _ in range(1500):
        G, B = rng.randint(2, 6), rng.randint(1, 6)
        report, gave_up_at, violations = _run_group(G, B, rng, p_give_up)
        if not gave_up_at:
            # (after a give-up the others may pass later barriers early: the
            # workgroup that gave up raises the counter without waiting; the
            # pair is then reported lost)
            assert not violations
        if any(g == 0 or b < B for g, b in gave_up_at):
            assert report == "lost"
        if p_give_up == 0.0:
            assert report == "ok" and not gave_up_at


def _run_pipeline(nb, G, rng, p_give_up):
    """The group elimination's pipeline (G >= 2 workgroups, nb row blocks of
    16 steps).  Row block bb belongs to workgroup 1 + bb mod (G - 1).
    Workgroup 0, for each block b: waits until the owner of b has published
    that it applied block b - 2 (b >= 2), applies block b - 1 itself (b >= 1),
    records b and publishes `recorded` = b + 1.  Owner g, for each b up to
    nb - 3: waits for `recorded` >= b + 1, applies block b to its blocks
    >= b + 2, publishes `applied[g]` = b + 1.  A wait may give up (then the
    workgroup stops waiting and sets its failure flag).  Returns the order
    in which each row block received the blocks' steps, the blocks whose
    record saw an incompletely updated row block, reads of unrecorded
    blocks, and the failure flags."""
    owner = lambda bb: 1 + bb % (G - 1)
    recorded = [0]
    applied = [0] * G
    got = [[] for _ in range(nb)]        # blocks applied to each row block, in order
    bad_record = []                      # (b, what the rows carried) when recorded too early
    bad_read = []                        # (g, b) applies of a block not yet recorded
    failed = [False] * G

    def wait(g, pred):
        while not failed[g] and not pred():
            if rng.random() < p_give_up:
                failed[g] = True
                break
            yield

    def wg0():
        for b in range(nb):
            if b >= 2:
                yield from wait(0, lambda: applied[owner(b)] >= b - 1)
            if b >= 1:
                got[b].append(b - 1)
            if got[b] != list(range(b)) and not any(failed):
                bad_record.append((b, list(got[b])))
            yield
            recorded[0] = b + 1
            yield

    def own(g):
        for b in range(nb - 2):
            yield from wait(g, lambda: recorded[0] >= b + 1)
            if recorded[0] < b + 1 and not failed[g]:
                bad_read.append((g, b))
            for bb in range(b + 2, nb):
                if owner(bb) == g:
                    got[bb].append(b)
                    yield
            applied[g] = b + 1
            yield

    procs = [wg0()] + [own(g) for g in range(1, G)]
    steps = 0
    while procs:
        p = rng.choice(procs)
        try:
            next(p)
        except StopIteration:
            procs.remove(p)
        steps += 1
        assert steps < 500000, "the model did not end"
    return got, bad_record, bad_read, failed


@pytest.mark.parametrize("p_give_up", [0.0, 0.01, 0.2])
def test_group_elimination_pipeline_orders_every_row_block(p_give_up):
    """Without a give-up every row block has received the steps of every
    earlier block, in order, when workgroup 0 records it, and no owner
    applies a block before it is recorded; every run ends, also when waits
    give up."""
    rng = random.Random(23)
    for _ in range(800):
        nb, G = rng.randint(1, 14), rng.randint(2, 9)
        got, bad_record, bad_read, failed = _run_pipeline(nb, G, rng, p_give_up)
        if not any(failed):
            assert not bad_record and not bad_read
            assert all(got[bb] == list(range(bb)) for bb in range(nb))
        if p_give_up == 0.0:
            assert not any(failed)
