"""Host logic of the real-time serving loop (paper_2211_16266_amd.serving),
without a GPU: a stand-in server that finishes each job after a given
number of ticks checks that requests are submitted only once they have
arrived and are ready, in arrival order; that latency counts from arrival
to the poll that sees the job done; that jobs are dropped after their
callback when asked; and the summary's counts."""
import time

from paper_2211_16266_amd import serving
from paper_2211_16266_amd._binding import Server


class FakeServer:
    TICK_S = 0.004

    def __init__(self):
        self.jobs = {}       # ticket -> ticks still to run
        self.submitted = []  # (ticket, job, time)
        self.ticks = 0
        self.occ = []

    def submit(self, job):
        tk = len(self.submitted)
        self.submitted.append((tk, job, time.perf_counter()))
        self.jobs[tk] = job["ticks"]
        return tk

    def step(self, stream=None):
        active = [tk for tk, n in self.jobs.items() if n > 0]
        if active:
            time.sleep(self.TICK_S)
            self.ticks += 1
            self.occ.append(len(active))
        for tk in active:
            self.jobs[tk] -= 1
        return len(active), 0

    def poll(self, tk):
        return Server.DONE if self.jobs[tk] == 0 else Server.RUNNING

    def stats(self):
        return {"mean_occupancy": sum(self.occ) / max(len(self.occ), 1), "ticks": self.ticks,
                "arena_peak": 0}


def test_arrivals_readiness_latency_and_summary():
    srv = FakeServer()
    done = []
    # request b depends on a (it starts from a's result); c is independent
    # (jobs are made at submission, as the loop does for anything that is
    # not a prepared job)
    reqs = [serving.Request(0.00, lambda: {"name": "a", "ticks": 10}, tag="a"),
            serving.Request(0.01, lambda: {"name": "b", "ticks": 3}, tag="b"),
            serving.Request(0.08, lambda: {"name": "c", "ticks": 2}, tag="c")]

    def ready(rq):
        return rq.tag != "b" or "a" in [t for t, _ in done]

    def on_done(rq, res):
        done.append((rq.tag, res))

    t0 = time.perf_counter()
    out = serving.run(srv, reqs, on_done=on_done, ready=ready, keep_jobs=False)
    assert [t for t, _ in done][0] == "a" and sorted(t for t, _ in done) == ["a", "b", "c"]
    names = [job["name"] for _, job, _ in srv.submitted]
    assert names.index("b") > names.index("a")
    res = {t: r for t, r in done}
    for tag, rq in zip("abc", reqs):
        r = res[tag]
        assert r.submit_s >= r.arrival_s - 1e-6
        assert r.done_s >= r.submit_s
        assert r.latency_s == r.done_s - r.arrival_s
        assert rq.job is None  # dropped after its callback
    # b waited for a: it was submitted no earlier than a was seen done
    assert res["b"].submit_s >= res["a"].done_s - 1e-6
    # every job ran its ticks, each tick taking at least TICK_S
    assert res["a"].latency_s >= 10 * FakeServer.TICK_S
    assert res["c"].submit_s >= 0.08 - 1e-6
    assert out["requests"] == 3 and len(out["results"]) == 3
    assert out["ticks"] == srv.ticks and out["p99_ms"] >= out["p50_ms"] > 0
    assert out["wall_s"] <= time.perf_counter() - t0


def test_empty_request_list_returns_at_once():
    srv = FakeServer()
    out = serving.run(srv, [])
    assert out["requests"] == 0 and out["results"] == [] and srv.submitted == []
