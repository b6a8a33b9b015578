#!/usr/bin/env python3
"""Emit csa_tree.inc: straight-line carry-save adder trees for bit-sliced
channel accumulation.

A 32-bit word here is a "bit-plane": bit b belongs to time sample b of a
32-sample group.  A 2-bit sample value v = lo + 2*hi contributes its lo plane
at weight 1 and its hi plane at weight 2.  The accumulator is NL planes
a[0..NL) holding, per bit position, a binary counter (a[L] has weight 2^L).

The emitted function csa_add_N<NL>(a, lo, hi) adds N channels.  Bits are
pushed level by level in streaming order: a level holds at most one pending
bit; a second bit arriving at that level is combined with the accumulator
and the pending bit by a full adder (carry-save adder, 3 bit-ops on 32
positions at once) whose carry is pushed one level up.  Left-over pending
bits are folded in with half adders at the end.  Sums never exceed
2^NL - 1, so the top level drops its (provably zero) carry.

Run:  python gen_csa.py > csa_tree.inc
"""
import sys

SIZES = (4, 8, 16, 32, 64)


class Emitter:
    def __init__(self, nl):
        self.nl = nl
        self.lines = []
        self.tmp = 0
        self.pending = [None] * nl

    def new(self):
        self.tmp += 1
        return f"t{self.tmp}"

    def full_add(self, level, x, y):
        """a[level] + x + y -> a[level] (sum), returns the carry name.
        Sum = xor3, carry = majority: one 3-input bit operation each."""
        cy = self.new()
        self.lines.append(f"  const uint32_t {cy} = BS_MAJ3(a[{level}], {x}, {y});")
        self.lines.append(f"  a[{level}] = BS_XOR3(a[{level}], {x}, {y});")
        return cy

    def half_add(self, level, x):
        cy = self.new()
        self.lines.append(f"  const uint32_t {cy} = a[{level}] & {x};")
        self.lines.append(f"  a[{level}] ^= {x};")
        return cy

    def push(self, level, x):
        if level == self.nl - 1:
            # top level: the carry out is zero by the range bound
            if self.pending[level] is None:
                self.pending[level] = x
            else:
                p = self.pending[level]
                self.pending[level] = None
                self.lines.append(f"  a[{level}] ^= {p} ^ {x};")
            return
        if self.pending[level] is None:
            self.pending[level] = x
            return
        p = self.pending[level]
        self.pending[level] = None
        cy = self.full_add(level, p, x)
        self.push(level + 1, cy)

    def flush(self):
        for level in range(self.nl):
            p = self.pending[level]
            if p is None:
                continue
            self.pending[level] = None
            if level == self.nl - 1:
                self.lines.append(f"  a[{level}] ^= {p};")
            else:
                cy = self.half_add(level, p)
                self.push(level + 1, cy)


class FastEmitter(Emitter):
    """Low counter of FAST levels only: a bit pushed to level FAST is the
    chunk's carry-out, returned instead of rippled further.  The low counter
    holds at most 2^FAST - 1 and a chunk of n channels adds at most 3 n;
    while their sum stays below 2^(FAST+1), at most one carry bit per
    position leaves the low counter, so the carry-out planes the tree makes
    are disjoint and merge with XOR."""

    def __init__(self, fast):
        super().__init__(fast + 1)
        self.fast = fast
        self.outs = []

    def push(self, level, x):
        if level == self.fast:
            self.outs.append(x)
            return
        if self.pending[level] is None:
            self.pending[level] = x
            return
        p = self.pending[level]
        self.pending[level] = None
        cy = self.full_add(level, p, x)
        self.push(level + 1, cy)

    def flush(self):
        for level in range(self.fast):
            p = self.pending[level]
            if p is None:
                continue
            self.pending[level] = None
            cy = self.half_add(level, p)
            self.push(level + 1, cy)


FAST = 5          # levels of the low counter
FAST_SIZES = (4, 8)


def emit_fast(n):
    assert 3 * n + 2 ** FAST - 1 < 2 ** (FAST + 1), "one carry-out per chunk"
    e = FastEmitter(FAST)
    for c in range(n):
        e.push(0, f"lo[{c}]")
        e.push(1, f"hi[{c}]")
    e.flush()
    outs = e.outs
    ret = outs[0] if outs else "0u"
    for o in outs[1:]:
        ret = f"({ret} ^ {o})"
    head = (f"template <int NL>\nstatic __host__ __device__ __forceinline__ uint32_t csa{FAST}_add_{n}"
            f"(uint32_t (&a)[NL], const uint32_t (&lo)[{n}], const uint32_t (&hi)[{n}])\n{{")
    return "\n".join([head] + e.lines + [f"  return {ret};", "}\n"])


def emit(n, nl):
    e = Emitter(nl)
    for c in range(n):
        e.push(0, f"lo[{c}]")
        e.push(1, f"hi[{c}]")
    e.flush()
    head = (f"static __host__ __device__ __forceinline__ void csa_add_{n}_{nl}"
            f"(uint32_t (&a)[{nl}], const uint32_t (&lo)[{n}], const uint32_t (&hi)[{n}])\n{{")
    return "\n".join([head] + e.lines + ["}\n"])


def main():
    out = ["// Generated by gen_csa.py -- do not edit.",
           "// Bit-sliced carry-save accumulation of 2-bit samples (see gen_csa.py).",
           "#pragma once", "#include <stdint.h>", ""]
    for nl in (12, 16):
        for n in SIZES:
            out.append(emit(n, nl))
    out.append(f"// Low-counter trees: add n channels into levels 0..{FAST - 1} of a[] and")
    out.append(f"// return the carry-out plane of weight 2^{FAST} (see FastEmitter).")
    for n in FAST_SIZES:
        out.append(emit_fast(n))
    sys.stdout.write("\n".join(out))


if __name__ == "__main__":
    main()
