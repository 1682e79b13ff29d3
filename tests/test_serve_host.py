"""Scheduling logic of the request server (host only): a stand-in batch with the
adg.Batch interface and a virtual clock, no GPU."""
import numpy as np

from paper_2501_01747_amd.serve import Request, Server, summarize

NOMEM = -2


class NoRoom(Exception):
    def __init__(self):
        super().__init__("no room")
        self.code = NOMEM


class FakeBatch:
    """Capacity in elements; a step costs `cost` virtual seconds per active element."""

    def __init__(self, capacity, slots, clock, cost=1e-4):
        self.capacity, self.used, self.clock, self.cost = capacity, 0, clock, cost
        self.E = [0] * slots
        self.target = [0] * slots
        self.done = [-1] * slots
        self.added = []
        self.max_step_past_target = 0

    def add(self, case, w0, n_steps=0):
        E = case["disc"]["n_elem"]
        if self.used + E > self.capacity:
            raise NoRoom()
        slot = self.done.index(-1) if -1 in self.done else None
        if slot is None:
            raise NoRoom()
        self.used += E
        self.E[slot], self.target[slot], self.done[slot] = E, n_steps, 0
        self.added.append(case["rid"])
        return slot

    def remove(self, slot):
        self.used -= self.E[slot]
        self.done[slot] = -1

    def step(self, n):
        for s in range(len(self.done)):
            if self.done[s] >= 0:
                self.done[s] = min(self.target[s], self.done[s] + n)
        self.clock.t += n * self.cost * self.used

    def poll(self):
        return np.array(self.done), np.zeros(len(self.done), dtype=np.int32)

    def state(self, slot):
        return np.full(3, float(self.done[slot]))


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


def case(rid, E):
    return {"rid": rid, "disc": {"n_elem": E, "order_p": 1}, "physics": {"n_species": 2}}


def test_every_request_completes_with_its_steps():
    clk = Clock()
    b = FakeBatch(1000, 8, clk)
    rng = np.random.default_rng(0)
    reqs = [Request(i, case(i, int(rng.integers(50, 400))), None, int(rng.integers(5, 50)), arrival=0.01 * i)
            for i in range(40)]
    res = Server(b, chunk=7, keep_states=True, clock=clk, sleep=clk.sleep).run(reqs)
    assert [r.rid for r in res] == list(range(40))
    for q, r in zip(reqs, res):
        assert r.ok and r.steps == q.steps and r.state[0] == q.steps
        assert r.arrival <= r.admitted <= r.completed
    s = summarize(res)
    assert s["completed_ok"] == 40 and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_admission_is_fifo_and_waits_for_space():
    clk = Clock()
    b = FakeBatch(500, 16, clk)
    sizes = [400, 300, 50, 450, 20]
    reqs = [Request(i, case(i, E), None, 10, arrival=0.0) for i, E in enumerate(sizes)]
    res = Server(b, chunk=4, clock=clk, sleep=clk.sleep).run(reqs)
    assert b.added == [0, 1, 2, 3, 4]          # no overtaking, even where a later request would fit
    adm = [r.admitted for r in res]
    assert adm == sorted(adm) and adm[1] > adm[0]


def test_request_larger_than_the_batch_fails_alone():
    clk = Clock()
    b = FakeBatch(100, 4, clk)
    res = Server(b, clock=clk, sleep=clk.sleep).run([Request(0, case(0, 500), None, 5),
                                                     Request(1, case(1, 50), None, 5, arrival=1.0)])
    assert not res[0].ok and res[1].ok and summarize(res)["failed"] == 1


def test_rounds_never_pass_the_nearest_target():
    clk = Clock()
    b = FakeBatch(1000, 4, clk)
    seen = []
    orig = b.step

    def step(n):
        seen.append(n)
        orig(n)

    b.step = step
    Server(b, chunk=10, clock=clk, sleep=clk.sleep).run([Request(0, case(0, 10), None, 13),
                                                         Request(1, case(1, 10), None, 25)])
    assert seen == [10, 3, 10, 2]
