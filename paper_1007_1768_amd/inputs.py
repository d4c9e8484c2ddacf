"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only builds inputs: reaction networks (reactant / product coefficient
matrices, rate constants, initial counts), time grids, loss weights and targets.  It holds
none of the simulation's arithmetic and imports neither the compiled library nor the
CPU oracle, so both sides can be fed the very same arrays.

Workloads (the paper's only model is its HIV network; these synthetic networks stand in
for it, with the shapes named in the workload list of the design notes):
  * immigration-death: 0 -> X (c = 10), X -> 0 (c = 0.1), X0 = 0, t_end = 100,
    101-point grid, 1,000 trajectories;
  * viral: T, I, V, E with x0 = (1000, 0, 100, 50), nine mass-action reactions,
    t_end = 50, 1,000-point grid, 10^4 trajectories;
  * random batch: 64 random mass-action networks (5-40 species, 10-120 uni- and
    bimolecular reactions, log-uniform rates in [1e-3, 1e1], initial counts in
    [10, 1000], t_end in [10, 100], 256-16,384 trajectories each, 200-point grids);
  * differentiated: the viral network at 10^5 trajectories with a squared-error loss
    against the means of the same model run with log-rates perturbed by N(0, 0.1^2);
  * large: the viral network, 10^6 trajectories, 10^4-point grid, 64-bin histogram of
    I per grid point, with the gradient;
  * wide networks (wide_network): 512-4096 reactions summed in the 64-chunk order, for
    the one-trajectory-per-wave kernels.
"""
import numpy as np


def _model(name, species, reactions, x0):
    """reactions: list of (reactant dict, product dict, rate)."""
    idx = {s: i for i, s in enumerate(species)}
    S, M = len(species), len(reactions)
    reac = np.zeros((M, S), dtype=np.int32)
    prod = np.zeros((M, S), dtype=np.int32)
    rates = np.zeros(M, dtype=np.float64)
    for j, (r, p, c) in enumerate(reactions):
        for s, v in r.items():
            reac[j, idx[s]] += v
        for s, v in p.items():
            prod[j, idx[s]] += v
        rates[j] = c
    return dict(name=name, species=list(species), reac=reac, prod=prod, rates=rates,
                x0=np.asarray(x0, dtype=np.int32))


def immigration_death(birth=10.0, death=0.1, x0=0):
    return _model("immigration_death", ["X"],
                  [({}, {"X": 1}, birth), ({"X": 1}, {}, death)], [x0])


VIRAL_SPECIES = ["T", "I", "V", "E"]


def viral(rates=None):
    base = [
        ({}, {"T": 1}, 10.0),                        # 0 -> T
        ({"T": 1}, {}, 0.01),                        # T -> 0
        ({"T": 1, "V": 1}, {"I": 1}, 2e-5),          # T + V -> I
        ({"I": 1}, {}, 0.5),                         # I -> 0
        ({"I": 1}, {"I": 1, "V": 1}, 20.0),          # I -> I + V
        ({"V": 1}, {}, 3.0),                         # V -> 0
        ({"I": 1, "E": 1}, {"E": 1}, 1e-3),          # I + E -> E
        ({"I": 1, "E": 1}, {"I": 1, "E": 2}, 1e-4),  # I + E -> I + 2E
        ({"E": 1}, {}, 0.1),                         # E -> 0
    ]
    m = _model("viral", VIRAL_SPECIES, base, [1000, 0, 100, 50])
    if rates is not None:
        m["rates"] = np.asarray(rates, dtype=np.float64).copy()
    return m


HIV_SPECIES = ["U0", "U", "T", "F", "Z4", "Z5", "I4", "I5", "V4", "V5"]


def hiv(delta_v=2.0):
    """The HIV network of the paper's Table 1 (27 reactions over 10 species) with the rates
    and initial state of Section 2.1 (time in days).  The infectivities depend on the
    tumour necrosis factor F: beta_R5 = clamp(beta - K F, 0, beta), beta_X4 = beta + K F,
    and gamma likewise (K = 1e-7); they are given as rate laws (species, slope, lo, hi) on
    top of the base constants beta = 4e-5 and gamma = 2e-5.  Bursting (I -> 200 V) consumes
    the infected cell; the V5 -> V4 mutation is the mass-action reaction of Table 1 (the
    paper's additional time trigger is not specified and not modelled)."""
    lam, d_uf, d_ut, d_uz, d_t, d_tf = 200.0, 1e-5, 0.129, 0.005, 0.01, 1e-5
    beta, gamma, K = 4e-5, 2e-5, 1e-7
    s1, s2, s3, d_iz, mu, pi_, d_i, d_z = 1e-4, 1e-3, 1e-4, 0.06, 2.5e-3, 200.0, 0.33, 0.01
    R = [
        ({"U0": 1}, {"U0": 1, "U": 1}, lam),
        ({"U": 1, "F": 1}, {"F": 1}, d_uf),
        ({"U": 1}, {"T": 1}, d_ut),
        ({"U": 1}, {"Z4": 1}, d_uz),
        ({"U": 1}, {"Z5": 1}, d_uz),
        ({"T": 1}, {}, d_t),
        ({"T": 1, "F": 1}, {"F": 1}, d_tf),
        ({"T": 1, "V5": 1}, {"I5": 1}, beta),            # 7: beta_R5
        ({"T": 1, "V4": 1}, {"I4": 1}, beta),            # 8: beta_X4
        ({"Z5": 1, "V5": 1}, {"I5": 1}, gamma),          # 9: gamma_R5
        ({"Z4": 1, "V4": 1}, {"I4": 1}, gamma),          # 10: gamma_X4
        ({"I5": 1}, {"I5": 1, "Z5": 1}, s2),
        ({"I4": 1}, {"I4": 1, "Z4": 1}, s2),
        ({"I5": 1, "Z5": 1}, {"U": 1, "I5": 1, "Z5": 1}, s1),
        ({"I4": 1, "Z4": 1}, {"U": 1, "I4": 1, "Z4": 1}, s1),
        ({"I5": 1, "Z5": 1}, {"Z5": 1}, d_iz),
        ({"I4": 1, "Z4": 1}, {"Z4": 1}, d_iz),
        ({"V5": 1}, {"V4": 1}, mu),
        ({"I5": 1}, {"V5": 200}, pi_),
        ({"I4": 1}, {"V4": 200}, pi_),
        ({"V4": 1}, {"F": 1, "V4": 1}, s3),
        ({"I5": 1}, {}, d_i),
        ({"I4": 1}, {}, d_i),
        ({"Z5": 1}, {}, d_z),
        ({"Z4": 1}, {}, d_z),
        ({"V5": 1}, {}, delta_v),
        ({"V4": 1}, {}, delta_v),
    ]
    x0 = [1, 200, 1000, 0, 250, 250, 0, 0, 0, 100]
    m = _model("hiv", HIV_SPECIES, R, x0)
    M = len(R)
    F = HIV_SPECIES.index("F")
    sp = np.full(M, -1, dtype=np.int32)
    slope, lo, hi = np.zeros(M), np.zeros(M), np.full(M, np.inf)
    for j, sign, cap in ((7, -1.0, beta), (8, 1.0, np.inf), (9, -1.0, gamma), (10, 1.0, np.inf)):
        sp[j], slope[j], lo[j], hi[j] = F, sign * K, 0.0, cap
    m["laws"] = dict(species=sp, slope=slope, lo=lo, hi=hi)
    return m


def uniform_grid(t_end, G):
    """t_g = (t_end * g) / (G - 1): one product, then one quotient, in binary64; the last
    point is t_end itself (the two roundings can otherwise put it one ulp above t_end)."""
    if G == 1:
        return np.array([float(t_end)])
    g = np.arange(G, dtype=np.float64)
    grid = (float(t_end) * g) / float(G - 1)
    grid[-1] = float(t_end)
    return grid


def random_networks(seed=20100701, count=64, G=200):
    """Random mass-action networks for the batched workload.

    Reactant sides are uni- or bimolecular.  Apart from inflows (0 -> X), every reaction
    lowers the total molecule count by at least one (X -> 0, X + Y -> Z, X + Y -> 0,
    2X -> Y, X + Y -> X), so the number of events per trajectory stays bounded by the
    initial total plus the inflow events, and counts cannot blow up.  Every species gets
    a degradation reaction when M >= S.
    """
    rng = np.random.default_rng(seed)
    nets = []
    for b in range(count):
        S = int(rng.integers(5, 41))
        M = int(rng.integers(10, 121))
        reac = np.zeros((M, S), dtype=np.int32)
        prod = np.zeros((M, S), dtype=np.int32)
        order = rng.permutation(S)
        j = 0
        for s in order[:min(S, M)]:
            reac[j, s] = 1
            j += 1
        kinds = ["inflow", "bind", "annih", "dimer", "catdeg", "uni"]
        probs = [0.10, 0.30, 0.10, 0.15, 0.20, 0.15]
        while j < M:
            k = kinds[int(rng.choice(len(kinds), p=probs))]
            a, c_, z = (int(v) for v in rng.integers(0, S, size=3))
            if k == "inflow":
                prod[j, a] = 1
            elif k == "uni":
                reac[j, a] = 1
            elif k == "dimer":
                reac[j, a] = 2
                prod[j, z] = 1
            else:
                if c_ == a:
                    c_ = (a + 1) % S
                reac[j, a] += 1
                reac[j, c_] += 1
                if k == "bind":
                    prod[j, z] = 1
                elif k == "catdeg":
                    prod[j, a] = 1
            j += 1
        rates = 10.0 ** rng.uniform(-3.0, 1.0, size=M)
        x0 = rng.integers(10, 1001, size=S).astype(np.int32)
        t_end = float(rng.uniform(10.0, 100.0))
        n_traj = int(rng.integers(256, 16385))
        net_seed = int(rng.integers(0, 2**63 - 1))
        nets.append(dict(name="random%02d" % b, species=["S%d" % s for s in range(S)], reac=reac, prod=prod,
                         rates=rates, x0=x0, t_end=t_end, n_traj=n_traj, grid=uniform_grid(t_end, G),
                         seed=net_seed))
    return nets


def wide_network(M, seed=20100702, S=None):
    """A mass-action network with many reactions (hundreds to 4096) for the 64-chunk order.

    S = min(1024, max(8, M // 4)) species unless given.  Every species degrades (the first
    S reactions); the rest are drawn as inflows (8 %), conversions X -> Y (30 %),
    bindings X + Y -> Z (25 %), dimerisations 2X -> Y (12 %), catalysed degradations
    X + Y -> X (15 %) and annihilations X + Y -> 0 (10 %).  Rates are log-uniform in
    [1e-2, 1]; bimolecular rates are divided by 20 (about the mean initial count, so
    first- and second-order reactions fire at comparable rates).  Initial counts are
    uniform in [5, 40].  Only inflows add molecules, so trajectories stay short.
    """
    rng = np.random.default_rng(seed + M)
    if S is None:
        S = min(1024, max(8, M // 4))
    reac = np.zeros((M, S), dtype=np.int32)
    prod = np.zeros((M, S), dtype=np.int32)
    bimol = np.zeros(M, dtype=bool)
    j = 0
    for s in range(min(S, M)):
        reac[j, s] = 1
        j += 1
    kinds = ["inflow", "conv", "bind", "dimer", "catdeg", "annih"]
    probs = [0.08, 0.30, 0.25, 0.12, 0.15, 0.10]
    while j < M:
        k = kinds[int(rng.choice(len(kinds), p=probs))]
        a, b, z = (int(v) for v in rng.integers(0, S, size=3))
        if b == a:
            b = (a + 1) % S
        if k == "inflow":
            prod[j, a] = 1
        elif k == "conv":
            reac[j, a] = 1
            prod[j, b] = 1
        elif k == "dimer":
            reac[j, a] = 2
            prod[j, z] = 1
            bimol[j] = True
        else:
            reac[j, a] = 1
            reac[j, b] = 1
            bimol[j] = True
            if k == "bind":
                prod[j, z] = 1
            elif k == "catdeg":
                prod[j, a] = 1
        j += 1
    rates = 10.0 ** rng.uniform(-2.0, 0.0, size=M)
    rates[bimol] /= 20.0
    x0 = rng.integers(5, 41, size=S).astype(np.int32)
    return dict(name="wide%d" % M, species=["S%d" % s for s in range(S)], reac=reac, prod=prod, rates=rates,
                x0=x0, sum_order="block64")


def perturbed_rates(model, seed, sigma=0.1):
    """Rates whose logarithms are the model's plus N(0, sigma^2) noise (the target model)."""
    rng = np.random.default_rng(seed)
    eps = rng.normal(0.0, sigma, size=model["rates"].shape[0])
    return np.exp(np.log(model["rates"]) + eps)


def loss_weights(mean, target):
    """w = dL/dmean for L = sum (mean - target)^2."""
    return 2.0 * (np.asarray(mean) - np.asarray(target))


# Named workloads: (model factory, n_traj, t_end, G, extras)
WORKLOADS = {
    "immigration_death": dict(model=immigration_death, n_traj=1000, t_end=100.0, G=101, seed=1),
    "viral": dict(model=viral, n_traj=10_000, t_end=50.0, G=1000, seed=2),
    "differentiated": dict(model=viral, n_traj=100_000, t_end=50.0, G=1000, seed=4, target_seed=44,
                           perturb_seed=404),
    "large": dict(model=viral, n_traj=1_000_000, t_end=50.0, G=10_000, seed=5, hist=(1, 0, 1, 64),
                  target_seed=55, perturb_seed=505),
}
