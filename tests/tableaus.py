"""Butcher tableaus (c, A, b) used by the tests.

eq2 and eq3 are the paper's second- and third-order cRKDG schemes
(Section 2.2, equations (eq:2) and (eq:3)); ssp2/ssp3 are the Butcher forms of
the SSP-RK2/3 methods (Section 3.2.1 and Section 4.1.1); rk4 is the classical
fourth-order method (Section 2.2 remark on Butcher form; Section 4); rk38 is
Kutta's 3/8 rule, a second four-stage fourth-order method used only to test
tableau independence in the linear case (Section 3.5.1 theorem 'equivalence');
rkf5 is the fifth-order Runge--Kutta--Fehlberg method the numerical section
pairs with k = 4 (Section 4): Fehlberg's six-stage 4(5) pair advanced with its
fifth-order weights (E. Fehlberg, NASA TR R-315, 1969).
"""
import numpy as np


def T(A, b, c):
    return (np.array(A, dtype=float), np.array(b, dtype=float), np.array(c, dtype=float))


FE = T([[0.0]], [1.0], [0.0])
EQ2 = T([[0, 0], [0.5, 0]], [0, 1], [0, 0.5])
EQ3 = T([[0, 0, 0], [1 / 3, 0, 0], [0, 2 / 3, 0]], [0.25, 0, 0.75], [0, 1 / 3, 2 / 3])
SSP2 = T([[0, 0], [1, 0]], [0.5, 0.5], [0, 1])
SSP3 = T([[0, 0, 0], [1, 0, 0], [0.25, 0.25, 0]], [1 / 6, 1 / 6, 2 / 3], [0, 1, 0.5])
RK4 = T([[0, 0, 0, 0], [0.5, 0, 0, 0], [0, 0.5, 0, 0], [0, 0, 1, 0]],
        [1 / 6, 1 / 3, 1 / 3, 1 / 6], [0, 0.5, 0.5, 1])
RK38 = T([[0, 0, 0, 0], [1 / 3, 0, 0, 0], [-1 / 3, 1, 0, 0], [1, -1, 1, 0]],
         [1 / 8, 3 / 8, 3 / 8, 1 / 8], [0, 1 / 3, 2 / 3, 1])
RKF5 = T([[0, 0, 0, 0, 0, 0],
          [1 / 4, 0, 0, 0, 0, 0],
          [3 / 32, 9 / 32, 0, 0, 0, 0],
          [1932 / 2197, -7200 / 2197, 7296 / 2197, 0, 0, 0],
          [439 / 216, -8, 3680 / 513, -845 / 4104, 0, 0],
          [-8 / 27, 2, -3544 / 2565, 1859 / 4104, -11 / 40, 0]],
         [16 / 135, 0, 6656 / 12825, 28561 / 56430, -9 / 50, 2 / 55],
         [0, 1 / 4, 3 / 8, 12 / 13, 1, 1 / 2])
