"""The paper's operation counts (oracle side), App. B.

Update step (App. B.1, table of multiplications; gamma is the cost of one
inverse square root): the row counts are
  y_bar               p*4 + p*36        S_inov          p
  S_cz                p*4*m             S_cz^T S_cz     m*p*m
  EVD                 m^3               Gamma^-1, ^-1/2 m + gamma*m
  S_cz^T S_inov       m*p               S_cz Q Gamma^-1 Q^T S_cz^T S_inov
                                                        m^2 + m + m^2 + p*m
  S_cz^T (...)        m*p               Z (...)         n*m
  Z Q sqrt(m-1) Gamma^-1/2 Q^T          m + m^2 + m^3 + n*m*m
and their total (m^2+m) n + (m^2+7m+41) p + 2m^3 + 3m^2 + (3+gamma) m.
Prediction (App. B.2): (3/2 m + 1) n multiplications and (5/2 m - 1) n
additions.  Table 1 quotes operations as multiplications plus additions, with
additions taken equal to multiplications for the update.
"""
from __future__ import annotations


def update_rows(m: int, n: int, p: int, gamma: int = 0) -> list[int]:
    """The rows of the update-step multiplication table, in order."""
    return [p * 4 + p * 36, p, p * 4 * m, m * p * m, m ** 3, m + gamma * m, m * p,
            m * m + m + m * m + p * m, m * p, n * m, m + m * m + m ** 3 + n * m * m]


def update_multiplications(m: int, n: int, p: int, gamma: int = 0) -> int:
    """Closed-form total of the update-step table."""
    return (m * m + m) * n + (m * m + 7 * m + 41) * p + 2 * m ** 3 + 3 * m * m + (3 + gamma) * m


def update_operations(m: int, n: int, p: int) -> int:
    """Table 1 'Update (1 domain)': multiplications plus as many additions."""
    return 2 * update_multiplications(m, n, p)


def prediction_operations(m: int, n: int) -> int:
    """Table 1 'Prediction': (3/2 m + 1) n mults + (5/2 m - 1) n adds = 4 m n."""
    return (3 * m * n) // 2 + n + (5 * m * n) // 2 - n
