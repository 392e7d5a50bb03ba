"""Integer CRT (Section 2.2) and Garner's mixed-radix conversion (Section 2.5).

* ``residues``: RNS decomposition x_i = X mod q_i.
* ``crt_compose``: Eq. (crt_composition), X = | sum x_i qhat_i [qhat_i^-1]_(q_i) |_Q.
* ``garner_digits``: the mixed-radix digits v_k of Eq. (garner_mrc), each computed as
  the nested expression of Section 2.5: start from x_k, and for j = 0..k-1 subtract
  v_j then multiply by c_(j,k)^-1 = [q_j^-1]_(q_k).
* ``garner``: X = v_0 + v_1 q_0 + v_2 q_0 q_1 + ... (Eq. garner_mrc).
"""
from __future__ import annotations


def residues(X: int, moduli) -> list[int]:
    return [X % q for q in moduli]


def crt_compose(x, moduli) -> int:
    Q = 1
    for q in moduli:
        Q *= q
    s = 0
    for xi, qi in zip(x, moduli):
        qhat = Q // qi
        s += int(xi) * qhat * pow(qhat % qi, -1, qi)
    return s % Q


def garner_digits(x, moduli) -> list[int]:
    v = []
    for k, qk in enumerate(moduli):
        t = int(x[k]) % qk
        for j in range(k):
            t = (t - v[j]) * pow(moduli[j], -1, qk) % qk
        v.append(t)
    return v


def garner(x, moduli) -> int:
    v = garner_digits(x, moduli)
    X, M = 0, 1
    for vk, qk in zip(v, moduli):
        X += vk * M
        M *= qk
    return X
