"""Pattern-based partitioning of k-mer sets (coex_partition_kmers): parts
within their state budget, every pattern in exactly one part, sorted order.
Runs on the CPU (the counts are checked on the GPU in test_gpu_parity)."""
import pytest

import synth


@pytest.fixture(scope="module")
def coex():
    import paper_1509_01506_amd as m
    return m


def test_parts_cover_and_fit(coex):
    kmers = synth.random_kmers(60, 1000, 12)
    with pytest.raises(coex.CoexError) as e:  # one automaton would be past the device tables
        coex.Dfa.kmers(kmers)
    assert e.value.name == "ETOOBIG"
    for budget in (0, 1023, 300, 4096):
        p = coex.Partition(kmers, max_states=budget)
        cap = budget or 1023
        seen = []
        firsts = []
        for i in range(p.n_parts):
            n_states, ids = p.part(i)
            assert n_states <= cap, (budget, i, n_states)
            seen += ids
            firsts.append(min(kmers[j] for j in ids))
            # a part's automaton is no larger than its patterns' trie
            trie = {k[:l] for k in (kmers[j] for j in ids) for l in range(1, len(k) + 1)}
            assert n_states <= len(trie) + 1
        assert sorted(seen) == list(range(len(kmers)))
        assert firsts == sorted(firsts)  # parts follow the sorted pattern order
        if budget == 4096:
            assert p.n_parts >= 2
        p.free()


def test_duplicates_budget_and_errors(coex):
    p = coex.Partition(["ACGT", "ACGT", "ACGA", "TTTT"], max_states=6)
    parts = [p.part(i) for i in range(p.n_parts)]
    assert sorted(i for _, ids in parts for i in ids) == [0, 1, 2, 3]
    assert all(n <= 6 for n, _ in parts)
    with pytest.raises(coex.CoexError):
        coex.Partition(["ACGTACGT"], max_states=5)  # one k-mer alone needs 9 states
    with pytest.raises(coex.CoexError):
        coex.Partition(["ACGX"])
    with pytest.raises(coex.CoexError):
        coex.Partition([])
