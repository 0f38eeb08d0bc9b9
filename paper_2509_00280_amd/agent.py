"""The learned layout search of Section III-C (Algorithm 1): a masked double DQN
over bit interleavings, with our GPU MTTKRP as the environment.

The environment state is the N x l(p) encoding matrix (Section III-C.1): entry
(n, t) is 1 when key bit t takes the next unused low bit of mode n.  An action
picks the mode for the next key bit; modes whose l(n) bits are placed are
masked, so every episode ends in a valid interleaving (one of the Eq. (1)
multinomial count).  Only the terminal state is rewarded, with the speedup of
its all-mode MTTKRP over the ALTO layout; that reward is cached per layout and,
once a small reward model predicts it well enough, used to filter encodings
that are not worth measuring.

Pieces and where the paper fixes them:
  * networks: two 3x3 convolutions with 16 and 32 feature maps over the
    encoding matrix, then two fully connected layers, one output per mode;
    hidden units proportional to N and l(p) (Fig. 4);
  * double DQN loss with a target network updated every tau episodes, one
    minibatch of l(p) transitions per episode from a prioritized replay buffer
    (Algorithm 1; Table II: gamma 0.99, buffer 1M, tau 100, Adam, learning
    rate 1e-3 -> 1e-4, epsilon 1.0 -> 0.1, at most 5000 episodes);
  * reward shaping: every transition of an episode gets log(speedup) / l(p)
    (uniform credit, Section III-D);
  * reward model: fully connected, two hidden layers, trusted for filtering
    once its mean relative error on 10 unseen samples is below 10 %; an
    encoding predicted no worse than the best reward minus the model's error
    margin is measured, any other takes the predicted reward (Section III-D);
  * elastic early stopping: stop when the best reward has not improved for w
    episodes, w shrinking with epsilon (Section III-D).

Readings where the paper gives no number (each a parameter): epsilon and the
learning rate decay geometrically per episode to their minimum at
``decay_episodes`` (default E_max / 2); the patience window is
w = ceil(E_max * epsilon) (w starts at E_max, as Algorithm 1 initialises it,
and shrinks in proportion to epsilon); hidden units N * l(p) (at least 32) in
the Q-network and the reward model; prioritized replay with exponent 0.6 and
importance weights annealed from 0.4 to 1; terminal transitions do not
bootstrap.

Host code only (NumPy); the environment calls the HIP library.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------- layers


def _im2col(x: np.ndarray) -> np.ndarray:
    """(B, C, H, W) -> (B*H*W, C*9) patches of a 3x3 'same' convolution."""
    B, C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    win = np.lib.stride_tricks.sliding_window_view(xp, (3, 3), axis=(2, 3))  # B, C, H, W, 3, 3
    return win.transpose(0, 2, 3, 1, 4, 5).reshape(B * H * W, C * 9)


def _col2im(dcols: np.ndarray, shape) -> np.ndarray:
    """Adjoint of _im2col."""
    B, C, H, W = shape
    d = dcols.reshape(B, H, W, C, 3, 3)
    dxp = np.zeros((B, C, H + 2, W + 2), dtype=dcols.dtype)
    for i in range(3):
        for j in range(3):
            dxp[:, :, i:i + H, j:j + W] += d[:, :, :, :, i, j].transpose(0, 3, 1, 2)
    return dxp[:, :, 1:H + 1, 1:W + 1]


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            m *= self.b1
            m += (1.0 - self.b1) * g
            v *= self.b2
            v += (1.0 - self.b2) * g * g
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


class QNet:
    """conv3x3(16) - ReLU - conv3x3(32) - ReLU - FC(H) - ReLU - FC(N) over an N x L matrix."""

    def __init__(self, N: int, L: int, hidden: int, rng: np.random.Generator):
        self.N, self.L, self.H = N, L, hidden

        def he(shape, fan_in):
            return (rng.standard_normal(shape) * math.sqrt(2.0 / fan_in)).astype(np.float64)

        self.params = [he((16, 9), 9), np.zeros(16), he((32, 16 * 9), 16 * 9), np.zeros(32),
                       he((32 * N * L, hidden), 32 * N * L), np.zeros(hidden),
                       he((hidden, N), hidden) * 0.1, np.zeros(N)]

    def copy_from(self, other: "QNet"):
        for p, q in zip(self.params, other.params):
            p[...] = q

    def forward(self, x: np.ndarray, keep: bool = False):
        """x: (B, N, L) -> Q values (B, N)."""
        W1, b1, W2, b2, W3, b3, W4, b4 = self.params
        B = x.shape[0]
        N, L = self.N, self.L
        x4 = x.reshape(B, 1, N, L).astype(np.float64)
        c1 = _im2col(x4)
        z1 = c1 @ W1.T + b1                       # B*N*L, 16
        a1 = np.maximum(z1, 0.0)
        a1_4 = a1.reshape(B, N, L, 16).transpose(0, 3, 1, 2)
        c2 = _im2col(a1_4)
        z2 = c2 @ W2.T + b2                       # B*N*L, 32
        a2 = np.maximum(z2, 0.0)
        f = a2.reshape(B, N, L, 32).transpose(0, 3, 1, 2).reshape(B, 32 * N * L)
        z3 = f @ W3 + b3
        a3 = np.maximum(z3, 0.0)
        q = a3 @ W4 + b4
        if keep:
            self._cache = (x4.shape, c1, z1, c2, z2, f, z3, a3)
        return q

    def backward(self, dq: np.ndarray):
        """Gradients of the parameters for dL/dq (after forward(keep=True))."""
        W1, b1, W2, b2, W3, b3, W4, b4 = self.params
        shape, c1, z1, c2, z2, f, z3, a3 = self._cache
        B, _, N, L = shape
        gW4 = a3.T @ dq
        gb4 = dq.sum(0)
        da3 = dq @ W4.T
        dz3 = da3 * (z3 > 0)
        gW3 = f.T @ dz3
        gb3 = dz3.sum(0)
        df = dz3 @ W3.T
        da2 = df.reshape(B, 32, N, L).transpose(0, 2, 3, 1).reshape(B * N * L, 32)
        dz2 = da2 * (z2 > 0)
        gW2 = dz2.T @ c2
        gb2 = dz2.sum(0)
        dc2 = dz2 @ W2
        da1 = _col2im(dc2, (B, 16, N, L)).transpose(0, 2, 3, 1).reshape(B * N * L, 16)
        dz1 = da1 * (z1 > 0)
        gW1 = dz1.T @ c1
        gb1 = dz1.sum(0)
        return [gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4]


class RewardModel:
    """Fully connected predictor of the terminal reward: flattened state -> H -> H -> 1."""

    def __init__(self, d_in: int, hidden: int, rng: np.random.Generator, lr: float = 1e-3):
        def he(shape, fan_in):
            return rng.standard_normal(shape) * math.sqrt(2.0 / fan_in)

        self.params = [he((d_in, hidden), d_in), np.zeros(hidden), he((hidden, hidden), hidden), np.zeros(hidden),
                       he((hidden, 1), hidden) * 0.1, np.zeros(1)]
        self.opt = Adam(self.params, lr=lr)
        self.rel_err = math.inf

    def forward(self, x: np.ndarray, keep: bool = False) -> np.ndarray:
        W1, b1, W2, b2, W3, b3 = self.params
        z1 = x @ W1 + b1
        a1 = np.maximum(z1, 0.0)
        z2 = a1 @ W2 + b2
        a2 = np.maximum(z2, 0.0)
        y = (a2 @ W3 + b3)[:, 0]
        if keep:
            self._cache = (x, z1, a1, z2, a2)
        return y

    def backward(self, dy: np.ndarray):
        W1, b1, W2, b2, W3, b3 = self.params
        x, z1, a1, z2, a2 = self._cache
        dy = dy[:, None]
        gW3 = a2.T @ dy
        gb3 = dy.sum(0)
        dz2 = (dy @ W3.T) * (z2 > 0)
        gW2 = a1.T @ dz2
        gb2 = dz2.sum(0)
        dz1 = (dz2 @ W2.T) * (z1 > 0)
        gW1 = x.T @ dz1
        gb1 = dz1.sum(0)
        return [gW1, gb1, gW2, gb2, gW3, gb3]

    def fit(self, X: np.ndarray, y: np.ndarray, epochs: int = 60):
        """Mean-squared error on log rewards, full batch."""
        t = np.log(y)
        for _ in range(epochs):
            p = self.forward(X, keep=True)
            self.opt.step(self.params, self.backward(2.0 * (p - t) / len(t)))

    def predict(self, X: np.ndarray) -> np.ndarray:
        return np.exp(self.forward(X))


class PrioritizedReplay:
    """Proportional prioritized replay (priorities |TD error| + 1e-3, exponent alpha)."""

    def __init__(self, capacity: int, alpha: float = 0.6):
        self.capacity, self.alpha = capacity, alpha
        self.data: list = []
        self.prio = np.zeros(capacity)
        self.pos = 0

    def __len__(self):
        return len(self.data)

    def add(self, item):
        p = self.prio[: len(self.data)].max() if self.data else 1.0
        if len(self.data) < self.capacity:
            self.data.append(item)
        else:
            self.data[self.pos] = item
        self.prio[self.pos] = p
        self.pos = (self.pos + 1) % self.capacity

    def sample(self, k: int, beta: float, rng: np.random.Generator):
        n = len(self.data)
        p = self.prio[:n] ** self.alpha
        p /= p.sum()
        idx = rng.choice(n, size=k, p=p)
        w = (n * p[idx]) ** (-beta)
        return idx, [self.data[i] for i in idx], w / w.max()

    def update(self, idx, td):
        self.prio[idx] = np.abs(td) + 1e-3


# ---------------------------------------------------------------- the search


def layout_to_state(layout, N: int) -> np.ndarray:
    s = np.zeros((N, len(layout)), dtype=np.float32)
    for t, n in enumerate(layout):
        s[int(n), t] = 1.0
    return s


def valid_actions(counts: np.ndarray, lbits: np.ndarray) -> np.ndarray:
    """Modes that still have an unplaced bit (the rule-driven action mask)."""
    return counts < lbits


@dataclass
class SearchResult:
    best_layout: list
    best_reward: float                 # speedup over ALTO of the best measured encoding
    episodes: int
    evaluations: int                   # real (measured) rewards
    cache_hits: int
    imagined: int                      # terminal rewards taken from the reward model
    model_trusted_at: int | None       # episode at which the reward model passed the accuracy bar
    stopped_early: bool
    seconds: float
    history: list = field(default_factory=list)  # (episode, reward, measured) per episode
    policy: "QNet | None" = None                  # the trained policy network


def greedy_layout(policy: QNet, lbits) -> list:
    """Roll the trained policy out without exploration (masked argmax at every step)."""
    lbits = np.asarray(lbits, dtype=np.int64)
    N, L = len(lbits), int(lbits.sum())
    s = np.zeros((N, L), dtype=np.float32)
    counts = np.zeros(N, dtype=np.int64)
    layout = []
    for t in range(L):
        q = policy.forward(s[None])[0]
        q[~valid_actions(counts, lbits)] = -np.inf
        a = int(np.argmax(q))
        s[a, t] = 1.0
        counts[a] += 1
        layout.append(a)
    return layout


def relate_search(reward_fn, lbits, episodes: int = 5000, seed: int = 0, gamma: float = 0.99,
                  buffer: int = 1_000_000, tau: int = 100, lr: float = 1e-3, lr_min: float = 1e-4,
                  eps: float = 1.0, eps_min: float = 0.1, decay_episodes: int | None = None,
                  model_accuracy: float = 0.90, model_warmup: int = 20, max_evaluations: int | None = None,
                  hidden: int | None = None, log=None) -> SearchResult:
    """Algorithm 1.  reward_fn(layout) -> speedup over ALTO of that layout (a real
    measurement); lbits[n] = bits of mode n; layout[t] = mode of key bit t.
    ``max_evaluations`` bounds the real measurements (the search then stops)."""
    t_start = time.perf_counter()
    rng = np.random.default_rng(seed)
    lbits = np.asarray(lbits, dtype=np.int64)
    N, L = len(lbits), int(lbits.sum())
    if L == 0:
        return SearchResult([], 1.0, 0, 0, 0, 0, None, False, 0.0)
    H = hidden or max(32, N * L)
    policy = QNet(N, L, H, rng)
    target = QNet(N, L, H, rng)
    target.copy_from(policy)
    opt = Adam(policy.params, lr=lr)
    per = PrioritizedReplay(buffer)
    model = RewardModel(N * L, H, rng)
    decay_episodes = decay_episodes or max(1, episodes // 2)
    kappa = (eps_min / eps) ** (1.0 / decay_episodes)
    kappa_lr = (lr_min / lr) ** (1.0 / decay_episodes)
    cache: dict = {}
    samples_x: list = []
    samples_y: list = []
    best_layout, best = None, -math.inf
    since_best = 0
    evals = hits = imagined = 0
    trusted_at = None
    history = []
    stopped = False
    ep = 0
    for ep in range(1, episodes + 1):
        s = np.zeros((N, L), dtype=np.float32)
        counts = np.zeros(N, dtype=np.int64)
        memory = []
        layout = []
        for t in range(L):
            mask = valid_actions(counts, lbits)
            if rng.random() < eps:
                a = int(rng.choice(np.flatnonzero(mask)))
            else:
                q = policy.forward(s[None])[0]
                q[~mask] = -np.inf
                a = int(np.argmax(q))
            s2 = s.copy()
            s2[a, t] = 1.0
            counts[a] += 1
            layout.append(a)
            memory.append([s, a, 0.0, s2, t == L - 1])
            s = s2
        # FILTER_EXE_ACTION on the terminal action: cache, reward model, or a measurement
        key = tuple(layout)
        measured = False
        if key in cache:
            r = cache[key]
            hits += 1
            measured = True
        else:
            x = s.reshape(1, -1).astype(np.float64)
            use_model = model.rel_err < 1.0 - model_accuracy
            pred = float(model.predict(x)[0]) if use_model else None
            if pred is not None and best > 0 and pred < best * (1.0 - model.rel_err):
                r = pred
                imagined += 1
            else:
                r = float(reward_fn(list(layout)))
                cache[key] = r
                evals += 1
                measured = True
                samples_x.append(x[0])
                samples_y.append(r)
                # retrain the reward model; its error is measured on the 10 newest
                # samples, unseen in that training
                if len(samples_y) >= model_warmup:
                    X = np.asarray(samples_x)
                    Y = np.asarray(samples_y)
                    model.fit(X[:-10], Y[:-10])
                    p = model.predict(X[-10:])
                    model.rel_err = float(np.mean(np.abs(p - Y[-10:]) / Y[-10:]))
                    if model.rel_err < 1.0 - model_accuracy and trusted_at is None:
                        trusted_at = ep
        history.append((ep, r, measured))
        # one minibatch of l(p) transitions (Algorithm 1: once the buffer holds one)
        if len(per) >= L:
            beta = min(1.0, 0.4 + 0.6 * ep / episodes)
            idx, batch, w = per.sample(L, beta, rng)
            S = np.stack([b[0] for b in batch])
            A = np.array([b[1] for b in batch])
            R = np.array([b[2] for b in batch])
            S2 = np.stack([b[3] for b in batch])
            D = np.array([b[4] for b in batch])
            q2_pol = policy.forward(S2)
            q2_tgt = target.forward(S2)
            cnt2 = S2.sum(axis=2)                                  # bits placed per mode
            q2_pol[cnt2 >= lbits[None, :]] = -np.inf               # masked at s'
            a2 = np.argmax(q2_pol, axis=1)
            y = R + np.where(D, 0.0, gamma * q2_tgt[np.arange(L), a2])
            q = policy.forward(S, keep=True)
            td = y - q[np.arange(L), A]
            dq = np.zeros_like(q)
            dq[np.arange(L), A] = -2.0 * w * td / L
            opt.step(policy.params, policy.backward(dq))
            per.update(idx, td)
        if ep % tau == 0:
            target.copy_from(policy)
        eps = max(eps_min, eps * kappa)
        opt.lr = max(lr_min, opt.lr * kappa_lr)
        window = math.ceil(episodes * eps)
        if measured and r > best:
            best, best_layout = r, list(layout)
            since_best = 0
        else:
            since_best += 1
        # reward shaping: uniform credit log(speedup) / l(p) to every action of the episode
        shaped = math.log(max(r, 1e-12)) / L
        for m in memory:
            m[2] = shaped
            per.add(tuple(m))
        if log and (ep % 50 == 0 or ep == 1):
            log(f"episode {ep}: reward {r:.4f} best {best:.4f} eps {eps:.3f} window {window} evals {evals} "
                f"model err {model.rel_err:.3f}")
        if since_best >= window:
            stopped = True
            break
        if max_evaluations is not None and evals >= max_evaluations:
            break
    return SearchResult(best_layout, best, ep, evals, hits, imagined, trusted_at, stopped,
                        time.perf_counter() - t_start, history, policy)


# ---------------------------------------------------------------- GPU environment


def gpu_environment(dims, coords, vals, factors, iters: int = 5, repeats: int = 3):
    """The TD environment of the search: reward(layout) = all-mode MTTKRP time
    of the ALTO layout / that of `layout`.  Each layout is encoded on the GPU,
    prepared under the default plan and timed with HIP events on the current
    stream: `iters` all-mode MTTKRPs per measurement, the median of `repeats`
    measurements (the paper times 100 iterations, median of 3).  coords:
    (N, nnz) device int32, vals: device float32, factors: device FP32
    (dims[n], R).

    Returns (reward_fn, alto_layout, alto_ms, lbits) with lbits[n] the key bits of mode n."""
    import torch

    from . import spt

    R = int(factors[0].shape[1])
    outs = [torch.empty((int(d), R), device=factors[0].device) for d in dims]

    def measure(layout):
        h = spt.encode(dims, coords, vals, layout=layout)
        try:
            h.prepare(R)
            for n in range(len(dims)):
                spt.mttkrp(h, factors, n, out=outs[n])
            times = []
            for _ in range(repeats):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(iters):
                    for n in range(len(dims)):
                        spt.mttkrp(h, factors, n, out=outs[n])
                e1.record()
                e1.synchronize()
                times.append(e0.elapsed_time(e1) / iters)
        finally:
            h.free()
        return float(np.median(times))

    h = spt.encode(dims, coords, vals)
    info = h.info()
    h.free()
    alto = list(info["layout"])
    lbits = [int(b) for b in info["lbits"][: len(dims)]]
    alto_ms = measure(alto)

    def reward(layout):
        return alto_ms / measure(layout)

    return reward, alto, alto_ms, lbits
