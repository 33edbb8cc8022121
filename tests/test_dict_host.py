"""Host logic of dictionary-encoded predicates (no GPU): every comparison of
a string column with a literal, folded into a comparison of the codes, keeps
exactly the rows the string comparison keeps (the oracle's dictionary and
lookup stand in for the library's)."""
import itertools

import numpy as np
import pytest
import torch

import oracle
from paper_2211_02753_amd import dictenc

OPS = {"<": lambda a, b: a < b, "<=": lambda a, b: a <= b, ">": lambda a, b: a > b,
       ">=": lambda a, b: a >= b, "==": lambda a, b: a == b, "!=": lambda a, b: a != b}


def test_literal_predicate_agrees_with_string_comparison(monkeypatch):
    words = [b"delta", b"alpha", b"charlie", b"bravo", b"alpha", b"echo", b"", b"bravo", b"zulu"]
    rows = dictenc.pad(words, 8).numpy()
    d, codes = oracle.dict_build(rows)

    def fake_lookup(dictionary, strs):
        pos, found = oracle.dict_lookup(dictionary.numpy(), strs.numpy())
        return torch.from_numpy(pos), torch.from_numpy(found)

    monkeypatch.setattr(dictenc, "lookup", fake_lookup)
    dt = torch.from_numpy(d)
    literals = [b"", b"a", b"alpha", b"alphab", b"bravo", b"c", b"echo", b"f", b"zulu", b"zz"]
    for lit, op in itertools.product(literals, OPS):
        cop, clit = dictenc.literal_predicate(dt, op, lit)
        want = [OPS[op](w, lit) for w in words]
        got = [OPS[cop](int(c), clit) for c in codes]
        assert got == want, (lit, op, cop, clit)


def test_pad_rejects_what_does_not_fit():
    assert dictenc.pad([b"ab", b""], 4).tolist() == [[97, 98, 0, 0], [0, 0, 0, 0]]
    with pytest.raises(ValueError):
        dictenc.pad([b"abcde"], 4)
    with pytest.raises(ValueError):
        dictenc.pad([b"a\x00b"], 4)
