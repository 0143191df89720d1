"""Structure-adaptive tile Cholesky (dense and active-column routes) on MI355X."""
