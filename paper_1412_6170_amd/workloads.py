"""Seeded synthetic workloads for the repeated k-NN join.

This module only draws inputs: positions per tick, the querying objects and
their k.  It holds none of the method's arithmetic, so both the GPU path and
the CPU oracle can be fed from it.

The paper's experiments use a third-party moving-objects generator with
uniform, Gaussian-hotspot and road-network datasets (Sec. 5); those are not
available, and these generators stand in for them with the same kinds of
distributions.  All coordinates are float32 in [0, 1) -- the unit square --
and clamping uses [0, 1 - 2^-24], 1 - 2^-24 being the largest float32 below
one.  Object ids are positions in the returned arrays and are a random
permutation with respect to space.

Workloads (sizes as used by the tests and the benchmark):

* ``uniform_10k``   -- 1 tick, 10,000 objects uniform in [0,1)^2, every
  object queries with k = 8.
* ``clustered_1m``  -- 10 ticks, 1,000,000 objects: 80% drawn from 16
  Gaussian clusters (sigma 0.01, centres uniform), 20% uniform; each tick
  every object moves by an independent uniform step in [-1e-4, 1e-4] per
  axis, clamped to the square; every object queries with k = 32.
* ``network_4m``    -- 20 ticks, 4,000,000 objects on a random graph of 2,000
  nodes (uniform in the square, each joined to its 3 nearest nodes), placed
  uniformly along the edges (edge chosen by length) and moving along them at
  1e-4 per tick, turning onto a random incident edge at nodes; each tick a
  fresh half of the objects queries, each with k drawn from {8, 16, 32, 64}.
  (Stands in for the paper's road-network dataset.)
* ``mixed_16m``     -- 100 ticks, 16,000,000 objects: 50% uniform, 50% in 64
  Gaussian clusters (sigma 0.005); random-walk step uniform in
  [-5e-5, 5e-5] per axis, clamped; every object queries with k = 128.
"""
import numpy as np

SEED = 14126170
CLAMP_HI = np.float32(1.0 - 2.0 ** -24)


def rng_for(workload_id, tick, stream=0):
    """Independent generator per (workload, tick, stream)."""
    return np.random.default_rng([SEED, int(workload_id), int(tick), int(stream)])


def clamp01(a):
    """Clamp float32 values to [0, 1 - 2^-24] in place and return them."""
    np.clip(a, np.float32(0.0), CLAMP_HI, out=a)
    return a


def uniform_points(n, rng):
    x = rng.random(n, dtype=np.float32)
    y = rng.random(n, dtype=np.float32)
    return x, y


def gaussian_mixture(n, n_clusters, sigma, frac_clustered, rng):
    """frac_clustered of the objects around n_clusters uniform centres with
    standard deviation sigma per axis (drawn in float64, rounded to float32,
    clamped), the rest uniform; returned in a random order."""
    n_cl = int(round(n * frac_clustered))
    centres = rng.random((n_clusters, 2))
    which = rng.integers(0, n_clusters, size=n_cl)
    pts = centres[which] + rng.normal(0.0, sigma, size=(n_cl, 2))
    xc = clamp01(pts[:, 0].astype(np.float32))
    yc = clamp01(pts[:, 1].astype(np.float32))
    xu, yu = uniform_points(n - n_cl, rng)
    x = np.concatenate([xc, xu])
    y = np.concatenate([yc, yu])
    perm = rng.permutation(n)
    return np.ascontiguousarray(x[perm]), np.ascontiguousarray(y[perm])


def random_step(x, y, step, rng):
    """Move every object by an independent uniform step in [-step, step] per
    axis (float32 addition), then clamp to the square."""
    dx = rng.uniform(-step, step, size=len(x)).astype(np.float32)
    dy = rng.uniform(-step, step, size=len(y)).astype(np.float32)
    nx = clamp01(x + dx)
    ny = clamp01(y + dy)
    return nx, ny


class Workload:
    """A named sequence of ticks; ``tick(t)`` returns (x, y, issuers, ks, k)
    where issuers None means every object queries and ks None means uniform
    k."""

    def __init__(self, name, wid, n, ticks, k, description):
        self.name = name
        self.wid = wid
        self.n = n
        self.ticks = ticks
        self.k = k
        self.description = description
        self._cache = {}

    def positions(self, t):
        raise NotImplementedError

    def tick(self, t):
        x, y = self.positions(t)
        return x, y, None, None, self.k


class UniformWorkload(Workload):
    def positions(self, t):
        if t not in self._cache:
            self._cache = {t: uniform_points(self.n, rng_for(self.wid, t))}
        return self._cache[t]


class ClusteredMovingWorkload(Workload):
    def __init__(self, name, wid, n, ticks, k, description, n_clusters, sigma,
                 frac_clustered, step):
        super().__init__(name, wid, n, ticks, k, description)
        self.n_clusters = n_clusters
        self.sigma = sigma
        self.frac_clustered = frac_clustered
        self.step = step
        self._last = None  # (t, x, y)

    def positions(self, t):
        if self._last is not None and self._last[0] == t:
            return self._last[1], self._last[2]
        if self._last is not None and self._last[0] < t:
            t0, x, y = self._last
        else:
            t0 = 0
            x, y = gaussian_mixture(self.n, self.n_clusters, self.sigma,
                                    self.frac_clustered, rng_for(self.wid, 0))
        for s in range(t0 + 1, t + 1):
            x, y = random_step(x, y, self.step, rng_for(self.wid, s))
        self._last = (t, x, y)
        return x, y


class NetworkWorkload(Workload):
    """Objects moving along the edges of a random planar-ish graph."""

    def __init__(self, name, wid, n, ticks, description, n_nodes=2000, degree=3,
                 speed=1e-4, query_frac=0.5, k_choices=(8, 16, 32, 64)):
        super().__init__(name, wid, n, ticks, max(k_choices), description)
        self.speed = speed
        self.query_frac = query_frac
        self.k_choices = np.asarray(k_choices, np.int32)
        rng = rng_for(wid, 0, 1)
        nodes = rng.random((n_nodes, 2))
        d2 = ((nodes[:, None, :] - nodes[None, :, :]) ** 2).sum(-1)
        np.fill_diagonal(d2, np.inf)
        near = np.argsort(d2, axis=1)[:, :degree]
        edges = {(min(a, b), max(a, b)) for a in range(n_nodes) for b in near[a]}
        self.edges = np.array(sorted(edges), np.int64)            # [E, 2]
        self.nodes = nodes
        seg = nodes[self.edges[:, 1]] - nodes[self.edges[:, 0]]
        self.length = np.sqrt((seg ** 2).sum(1))
        inc = [[] for _ in range(n_nodes)]
        for e, (a, b) in enumerate(self.edges):
            inc[a].append(e)
            inc[b].append(e)
        self.incident = [np.asarray(v, np.int64) for v in inc]
        # initial state: edge (by length), distance from its first node, direction
        r0 = rng_for(wid, 0, 2)
        p = self.length / self.length.sum()
        self.edge = r0.choice(len(self.edges), size=n, p=p)
        self.pos = r0.random(n) * self.length[self.edge]
        self.dir = np.where(r0.random(n) < 0.5, 1.0, -1.0)
        self._t = 0

    def _advance(self, t):
        rng = rng_for(self.wid, t, 3)
        left = np.full(self.n, self.speed)
        for _ in range(64):
            L = self.length[self.edge]
            target = np.where(self.dir > 0, L, 0.0)
            room = np.abs(target - self.pos)
            done = left <= room
            self.pos = np.where(done, self.pos + self.dir * left, target)
            left = np.where(done, 0.0, left - room)
            idx = np.nonzero(~done)[0]
            if len(idx) == 0:
                break
            # at a node: continue on a random incident edge
            node = np.where(self.dir[idx] > 0, self.edges[self.edge[idx], 1],
                            self.edges[self.edge[idx], 0])
            u = rng.random(len(idx))
            for j, (i, v) in enumerate(zip(idx, node)):
                choices = self.incident[v]
                e = choices[int(u[j] * len(choices))]
                self.edge[i] = e
                if self.edges[e, 0] == v:
                    self.pos[i], self.dir[i] = 0.0, 1.0
                else:
                    self.pos[i], self.dir[i] = self.length[e], -1.0

    def positions(self, t):
        if t < self._t:
            raise ValueError("network workload only moves forward in time")
        while self._t < t:
            self._t += 1
            self._advance(self._t)
        a = self.nodes[self.edges[self.edge, 0]]
        b = self.nodes[self.edges[self.edge, 1]]
        f = (self.pos / self.length[self.edge])[:, None]
        xy = a + (b - a) * f
        x = clamp01(xy[:, 0].astype(np.float32))
        y = clamp01(xy[:, 1].astype(np.float32))
        return x, y

    def tick(self, t):
        x, y = self.positions(t)
        rng = rng_for(self.wid, t, 4)
        nq = int(round(self.n * self.query_frac))
        issuers = np.sort(rng.choice(self.n, nq, replace=False)).astype(np.int32)
        ks = rng.choice(self.k_choices, nq).astype(np.int32)
        return x, y, issuers, ks, None


def uniform_10k():
    return UniformWorkload(
        "uniform_10k", 1, 10_000, 1, 8,
        "1 tick, 10,000 objects uniform in [0,1)^2, all query, k=8")


def clustered_1m(n=1_000_000, ticks=10):
    return ClusteredMovingWorkload(
        "clustered_1m" if n == 1_000_000 else "clustered_%d" % n, 2, n, ticks, 32,
        "%d ticks, %d objects: 80%% in 16 Gaussian clusters (sigma 0.01), 20%% uniform, "
        "uniform step in [-1e-4,1e-4]^2 per tick, all query, k=32" % (ticks, n),
        n_clusters=16, sigma=0.01, frac_clustered=0.8, step=1e-4)


def network_4m(n=4_000_000, ticks=20):
    return NetworkWorkload(
        "network_4m" if n == 4_000_000 else "network_%d" % n, 3, n, ticks,
        "%d ticks, %d objects moving along a random 2,000-node graph at 1e-4/tick, "
        "half of them query each tick with k in {8,16,32,64}" % (ticks, n))


def mixed_16m(n=16_000_000, ticks=100):
    return ClusteredMovingWorkload(
        "mixed_16m" if n == 16_000_000 else "mixed_%d" % n, 5, n, ticks, 128,
        "%d ticks, %d objects: 50%% uniform, 50%% in 64 Gaussian clusters (sigma 0.005), "
        "uniform step in [-5e-5,5e-5]^2 per tick, all query, k=128" % (ticks, n),
        n_clusters=64, sigma=0.005, frac_clustered=0.5, step=5e-5)


WORKLOADS = {"uniform_10k": uniform_10k, "clustered_1m": clustered_1m, "network_4m": network_4m,
             "mixed_16m": mixed_16m}
