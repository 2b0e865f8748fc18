"""The warm-start policy of the serving loop (serving.WarmStartServer), on the host: which resident
prior a request starts from, and what is kept resident.  Theorem 2 and Propositions 1-2 make a warm
start from a dominating prior exact, so such priors are preferred; any other prior is still
conservative (Theorem 1) and is used only when no dominating one is resident, unless the server
is told to start cold then.  No GPU: the context is never called by these methods."""
from paper_1903_07715_amd import hjr, serving


def _req(key, kind="dubins3"):
    # dominates(a, b): the prior a has at least the control bound and at most the disturbance of b
    return serving.Request(kind=kind, grid=None, dyn=None, key=key, dominates=lambda a, b: a[0] >= b[0] and a[1] <= b[1],
                           l_dev=None, opts={})


def _kept(srv, key, V, kind="dubins3"):
    r = _req(key, kind)
    r.V = V
    srv.keep(r)


def test_prefers_the_nearest_dominating_prior():
    srv = serving.WarmStartServer(ctx=None)
    _kept(srv, (2.0, 0.00), "far-dominating")
    _kept(srv, (1.6, 0.05), "near-dominating")
    _kept(srv, (1.4, 0.10), "nearest-but-weaker")   # less control: does not dominate (1.5, 0.1)
    V, key, exact = srv.pick_warm_start(_req((1.5, 0.10)))
    assert (V, key, exact) == ("near-dominating", (1.6, 0.05), True)


def test_falls_back_to_the_nearest_prior_or_starts_cold():
    srv = serving.WarmStartServer(ctx=None)
    _kept(srv, (1.0, 0.20), "weak")
    _kept(srv, (1.2, 0.15), "less-weak")
    V, key, exact = srv.pick_warm_start(_req((1.5, 0.10)))
    assert (V, key, exact) == ("less-weak", (1.2, 0.15), False)
    strict = serving.WarmStartServer(ctx=None, only_dominating=True)
    strict.resident = srv.resident
    assert strict.pick_warm_start(_req((1.5, 0.10))) == (None, None, None)
    cold = serving.WarmStartServer(ctx=None, warm=False)
    cold.resident = srv.resident
    assert cold.pick_warm_start(_req((1.5, 0.10))) == (None, None, None)


def test_priors_of_another_kind_are_not_used():
    srv = serving.WarmStartServer(ctx=None)
    _kept(srv, (2.0, 0.0), "quad", kind="quad6")
    assert srv.pick_warm_start(_req((1.5, 0.1))) == (None, None, None)


def test_keeps_the_most_recently_used_priors_per_kind():
    srv = serving.WarmStartServer(ctx=None, resident_per_kind=2)
    _kept(srv, (1.0, 0.1), "a")
    _kept(srv, (1.1, 0.1), "b")
    assert srv.pick_warm_start(_req((1.05, 0.15)))[0] == "b"   # b is now the latest use
    _kept(srv, (1.2, 0.1), "c")                    # evicts a, the least recently used
    assert sorted(c[1] for c in srv.resident["dubins3"]) == ["b", "c"]


def test_latency_stats_count_only_converged_results():
    reqs = []
    for i, st in enumerate([hjr.OK, hjr.OK, hjr.NOT_CONVERGED, hjr.OK]):
        r = _req((1.0, 0.1))
        r.arrival, r.done, r.status = float(i), float(i) + 0.5 * (i + 1), st
        reqs.append(r)
    s = serving.latency_stats(reqs)
    assert (s["requests"], s["converged"], s["not_converged"]) == (4, 3, 1)
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    assert abs(s["solves_per_s"] - 3 / span) < 1e-12
    assert s["p50_s"] == 1.0 and s["p99_s"] == 2.0
