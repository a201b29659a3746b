"""Inputs shared by the oracle pins and the GPU tests of the estimator's
rarely taken branches (plain data; no arithmetic of the method)."""

# The truncation max{1, E^ML[Y]} of eq:gradient_estimator (Sec. 2.2) fires:
# the target is scaled up and the control undershoots it, so the coarse
# partner of a level (full weighting shrinks the data) misses the target by
# more than the fine solve; at theta = 3 the negative level corrections then
# outweigh level 0 and E^ML[Y] is far below 1 (about -3e3 on these draws).
TRUNCATION_CASE = {"grid": [5, 9, 17], "M": [2, 2, 1], "first": [2, 3, 0], "theta": 3.0,
                   "alpha": 1e-3, "seed": 0, "yd_scale": 20.0, "u_over_yd": 0.7 * 29.0}

# The level update of eq:optimal-level (Sec. 4.1) adds a level: a control
# close to the optimum 15.8 y_d (sigma = 1, alpha = 1e-3) makes eps = 0.9 |g|
# small, so the squared-bias estimate of two levels on a three-level grid
# list exceeds eps^2 / 2 (by a factor of about 2).
LEVEL_GROWTH_CASE = {"grid": [9, 17, 33], "M": [16, 8], "theta": 1.0, "alpha": 1e-3,
                     "sigma2": 1.0, "u_over_yd": 15.8}
