"""Property test (hypothesis): on random connected graphs of up to 40 nodes,
CPU Greedy++ (pruned BFS, lazy skip, any block schedule) picks exactly what
the plain greedy by definition picks; the plain greedy checks its own
invariants (F = sum of d(S,.), d(S,.) and gains never increase, the farness
drop equals the pick's gain) as it runs."""
from hypothesis import given, settings, strategies as st

import graphgen
import oracle


@settings(max_examples=60, deadline=None)
@given(n=st.integers(2, 40), p=st.floats(0.02, 0.5), seed=st.integers(0, 10**6),
       kfrac=st.floats(0.0, 1.0), block=st.integers(1, 70), growth=st.integers(1, 8))
def test_tier_b_equals_tier_a_on_random_graphs(n, p, seed, kfrac, block, growth):
    g = graphgen.gnp_connected(n, p, seed)
    k = max(1, min(g.n, int(round(kfrac * g.n))))
    grp_a, F_a = oracle.greedy(g, k)
    grp_b, F_b, ev, _ = oracle.greedypp(g, k, block=block, growth=growth)
    assert grp_a.tolist() == grp_b.tolist()
    assert F_a.tolist() == F_b.tolist()
    assert int(ev[0]) == 0 and (k < 2 or int(ev[1]) == g.n - 1)
