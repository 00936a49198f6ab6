"""Offline stage end to end (Algorithm 2 with the rounding step of the GPU
path): cross on f_kappa, TT-Round and gauge of the small cores, then Phase 3
on the points.  Test infrastructure only."""
from . import cross, kernels, pttk


def offline(problem: kernels.Problem, X, Y, eps, seed=0, max_rank=256, max_sweeps=200,
            init_card=2, init_max_it=10, n_test=None, round_eps=None, forced=None):
    ent = cross.Entries(problem.entries, problem.n)
    cores, info = cross.greedy_cross(ent, eps, seed=seed, max_rank=max_rank,
                                     max_sweeps=max_sweeps, init_card=init_card,
                                     init_max_it=init_max_it, n_test=n_test, forced=forced)
    d, dt = problem.d, problem.dt
    G = pttk.round_and_gauge(cores, eps if round_eps is None else round_eps, d, dt)
    ns = problem.n[0]
    U = pttk.factor_values(X, problem.box_s, ns)
    V = pttk.factor_values(Y, problem.box_t, ns)
    S = pttk.phase3_source(U, G[:d])
    T = pttk.phase3_target(V, G[d + dt:])
    return {"S": S, "T": T, "param": G[d:d + dt], "cores": G, "cross_cores": cores,
            "info": info, "ranks": [1] + [g.shape[2] for g in G]}
