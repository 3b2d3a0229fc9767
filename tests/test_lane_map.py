"""CPU model of which device elements one step launch writes.

The step kernel walks the chunk list with a grid of G blocks: physical block
b takes logical position lb = logical_block(b) (runs of 32 consecutive
chunks per XCD when G is a multiple of 256, else lb = b), then chunks lb,
lb + G, lb + 2G, ...  Lane l of chunk c stands for node c * 256 + l; lanes
past the list load node nf - 1 but store to their own padded slot, element
(c, i, l), in both the next state and the full-way delay line.  The model
below replays that map for many (nf, G) and checks that no two lanes of a
launch write the same element and that every node's slots are written by
its own lane."""
import numpy as np
import pytest

CHUNK = 256
XCD_RUN = 32


def logical_block(b, G):
    if G % (8 * XCD_RUN) != 0:
        return b
    xcd, j = b & 7, b >> 3
    return ((j // XCD_RUN) * 8 + xcd) * XCD_RUN + j % XCD_RUN


def writes(nf, G, S):
    """(element, writer node or -1 for a padded lane) of every store of one launch."""
    chunks = (nf + CHUNK - 1) // CHUNK
    el, who = [], []
    lanes = np.arange(CHUNK)
    for b in range(G):
        c = logical_block(b, G)
        while c < chunks:
            n = c * CHUNK + lanes
            live = n < nf
            for i in range(S):
                el.append(c * S * CHUNK + i * CHUNK + lanes)   # slot = lane, not n % 256 of the clamped node
                who.append(np.where(live, n, -1))
            c += G
    return np.concatenate(el), np.concatenate(who)


def node_elem(n, i, S):
    return (n // CHUNK) * S * CHUNK + i * CHUNK + n % CHUNK


@pytest.mark.parametrize("nf", [1, 70, 255, 256, 257, 1000, 65536 + 70, 300001])
@pytest.mark.parametrize("G", [1, 8, 24, 256, 512, 1280])
@pytest.mark.parametrize("S", [19, 20])
def test_every_element_has_one_writer(nf, G, S):
    chunks = (nf + CHUNK - 1) // CHUNK
    G = min(G, chunks)
    el, who = writes(nf, G, S)
    assert len(np.unique(el)) == len(el), "two lanes store to one element"
    assert el.max() < chunks * S * CHUNK, "a store past the padded state"
    live = who >= 0
    n = who[live]
    i = (el[live] // CHUNK) % S
    assert np.array_equal(el[live], node_elem(n, i, S)), "a node's value stored outside its slot"
    assert live.sum() == nf * S


@pytest.mark.parametrize("G", [256, 512, 768, 1280, 2048])
def test_logical_block_is_a_bijection(G):
    lbs = [logical_block(b, G) for b in range(G)]
    assert sorted(lbs) == list(range(G))
