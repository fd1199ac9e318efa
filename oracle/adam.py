"""Adam (Kingma and Ba, ICLR 2015), the first-order optimiser the paper
trains every INR with (Sec. IV; hyper-parameters not given in the paper).

Reading: beta1 = 0.9, beta2 = 0.999, eps = 1e-8, no weight decay, bias
correction as in the original algorithm:
  m <- b1 m + (1 - b1) g ;  v <- b2 v + (1 - b2) g^2
  theta <- theta - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
with t the 1-based step count.
"""
import numpy as np


def adam_update(theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    theta = np.asarray(theta, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
