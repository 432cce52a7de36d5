"""The paper's Dslash cost model (Sec. 5.1), re-derived from the stencil's shape."""
import os

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "dslash_cost_model.txt")


def load():
    out = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def test_counts_follow_from_the_stencil():
    g = load()
    matvecs = 4 * 4                      # 4 directions x (+1, -1, +3, -3)
    cmul, cadd = 6, 2                    # real FLOP per complex multiply / add
    matvec_flop = 9 * cmul + 6 * cadd    # 3x3 complex matrix times 3-vector
    vec_adds = matvecs - 1               # summing 16 colour vectors
    assert matvecs * matvec_flop + vec_adds * 3 * cadd == g["flop_per_site"]
    assert matvecs * 18 == g["link_words_per_site"]
    assert matvecs * 6 == g["vector_words_read_per_site"]
    assert 6 == g["vector_words_written_per_site"]
    words = g["link_words_per_site"] + g["vector_words_read_per_site"] + g["vector_words_written_per_site"]
    # the paper quotes these "about" to two digits (0.367 is printed as 0.36)
    assert abs(g["flop_per_site"] / (4 * words) - g["ai_fp32_flop_per_byte"]) < 0.01
    assert abs(g["flop_per_site"] / (8 * words) - g["ai_fp64_flop_per_byte"]) < 0.01
