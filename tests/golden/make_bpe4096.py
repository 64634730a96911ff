"""Writes bpe4096_order5_64M.txt: the ranked merge table of the batched BPE
workload (4096 merges learned by the oracle's BPE trainer on 64 Mbase of the
seeded order-5 Markov genome of ``synth.bpe_corpus``). One merge per line,
"left right", rank = line number (0-based); merge r creates id 10 + r.

Calls only ``synth`` (inputs) and ``oracle`` (the trainer). About 30 s."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bpe4096_order5_64M.txt")


def make() -> np.ndarray:
    return oracle.bpe_train(synth.bpe_corpus(), 4096)


def save(merges, path=OUT):
    with open(path, "w") as f:
        for a, b in merges:
            f.write("%d %d\n" % (a, b))


def load(path=OUT) -> np.ndarray:
    return np.loadtxt(path, dtype=np.int32).reshape(-1, 2)


if __name__ == "__main__":
    save(make())
    print(OUT)
